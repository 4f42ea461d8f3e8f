"""FP64 CPU oracle for the spectral-element PCG solve (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
cpu_baseline leg of the benchmark may import this package; the product path
never does.  The C source (``oracle.c``) shares no code with the HIP library.

Every function here only marshals numpy arrays into the C library; the
arithmetic lives in ``oracle.c``, each step citing the passage it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CONVERGED, MAXITER, STAGNATED, BREAKDOWN = 1, 2, 3, 4
PC_IDENTITY, PC_JACOBI, PC_NN, PC_MG = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    lib.orc_gll.argtypes = [C.c_int, dp, dp]
    lib.orc_deriv.argtypes = [C.c_int, dp, dp]
    lib.orc_mesh_create.argtypes = [C.c_int, C.c_int, vp, vp, vp, vp, C.c_double,
                                    C.POINTER(vp)]
    lib.orc_mesh_destroy.argtypes = [vp]
    lib.orc_mesh_nloc.argtypes = [vp]
    lib.orc_mesh_nloc.restype = C.c_int64
    lib.orc_dot2_f32.argtypes = [C.c_int64, vp, vp]
    lib.orc_dot2_f32.restype = C.c_float
    lib.orc_dot_f32.argtypes = [C.c_int64, vp, vp]
    lib.orc_dot_f32.restype = C.c_float
    lib.orc_dot_c_f32.argtypes = [vp, C.c_int, vp, vp]
    lib.orc_dot_c_f32.restype = C.c_float
    lib.orc_gs_f32.argtypes = [vp, vp, C.c_int, C.c_int, vp]
    lib.orc_gs_f32.restype = C.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = C.c_int
    lib.orc_mesh_ngroups.argtypes = [vp]
    lib.orc_mesh_ngroups.restype = C.c_int64
    lib.orc_mesh_mindet.argtypes = [vp]
    lib.orc_mesh_mindet.restype = C.c_double
    lib.orc_mesh_get.argtypes = [vp, C.c_int, vp]
    for f in ("orc_ax_local", "orc_apply", "orc_rhs"):
        getattr(lib, f).argtypes = [vp, vp, vp]
    for f in ("orc_gs", "orc_mask", "orc_diag"):
        getattr(lib, f).argtypes = [vp, vp]
    lib.orc_dot.argtypes = [vp, vp, vp]
    lib.orc_dot.restype = C.c_double
    lib.orc_pcg.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int, C.c_double, C.c_int, vp,
                            vp]
    lib.orc_fcg.argtypes = [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int, vp, vp]
    lib.orc_ir.argtypes = [vp, C.c_int, vp, vp, C.c_double, C.c_double, C.c_int, C.c_int,
                           vp, vp]
    lib.orc_nn_create.argtypes = [C.c_int, C.c_int, vp, vp, C.POINTER(vp)]
    lib.orc_nn_destroy.argtypes = [vp]
    lib.orc_nn_set.argtypes = [vp, vp, vp]
    lib.orc_nn_local.argtypes = [vp, vp, vp, vp, vp]
    lib.orc_nn_apply.argtypes = [vp, vp, vp, vp]
    lib.orc_nn_loss_grad.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp]
    lib.orc_adam.argtypes = [C.c_int, vp, vp, vp, vp, C.c_int, C.c_double, C.c_double,
                             C.c_double, C.c_double]
    lib.orc_mg_create.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.POINTER(vp)]
    lib.orc_mg_destroy.argtypes = [vp]
    for f in ("orc_mg_apply", "orc_mg_schwarz_local", "orc_mg_restrict", "orc_mg_prolong_add"):
        getattr(lib, f).argtypes = [vp, vp, vp, vp]
    lib.orc_mg_nlev.argtypes = [vp]
    lib.orc_mg_level_nu.argtypes = [vp, C.c_int]
    lib.orc_mg_level_omega.argtypes = [vp, C.c_int]
    lib.orc_mg_level_omega.restype = C.c_double
    lib.orc_mg_level_dense.argtypes = [vp, C.c_int, vp]
    lib.orc_mg_vcycle.argtypes = [vp, vp, vp]
    lib.orc_mg_eig.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("reason", C.c_int), ("outer", C.c_int),
                ("fallback", C.c_int), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double)]


@dataclass
class SolveStats:
    iterations: int
    reason: int
    outer: int
    fallback: int
    rel_res_recursive: float
    rel_res_true: float


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1)


def dot2_f32(x, y) -> np.float32:
    """Dot2 (Ogita, Rump, Oishi 2005) of two FP32 vectors, in index order."""
    x, y = _f32(x), _f32(y)
    assert x.size == y.size
    return np.float32(_load().orc_dot2_f32(x.size, _p(x), _p(y)))


def dot_f32(x, y) -> np.float32:
    """Recursive FP32 dot in index order."""
    x, y = _f32(x), _f32(y)
    assert x.size == y.size
    return np.float32(_load().orc_dot_f32(x.size, _p(x), _p(y)))


def max_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_max_threads())


def gll(N: int):
    """GLL nodes and weights on [-1, 1] (ascending)."""
    lib = _load()
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    rc = lib.orc_gll(N, xi.ctypes.data_as(C.POINTER(C.c_double)),
                     w.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError(f"orc_gll({N}) failed: {rc}")
    return xi, w


def deriv(N: int) -> np.ndarray:
    """Nodal derivative matrix D[i, j] = l_j'(xi_i)."""
    lib = _load()
    xi, _ = gll(N)
    D = np.zeros((N + 1, N + 1))
    rc = lib.orc_deriv(N, xi.ctypes.data_as(C.POINTER(C.c_double)),
                       D.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError(rc)
    return D


class Mesh:
    """Oracle mesh: FP64 geometric factors, gather-scatter groups, mask, dinv."""

    def __init__(self, E: int, N: int, xyz, glo, bnd, kcoef=None, helm_h: float = 0.0):
        lib = _load()
        self.E, self.N, self.n = int(E), int(N), int(N) + 1
        self.nloc = self.E * self.n ** 3
        xyz = _f64(xyz)
        glo = np.ascontiguousarray(glo, dtype=np.int64)
        bnd = np.ascontiguousarray(bnd, dtype=np.uint8)
        assert xyz.size == 3 * self.nloc and glo.size == self.nloc and bnd.size == self.nloc
        kk = None if kcoef is None else _f64(kcoef)
        if kk is not None:
            assert kk.size == self.nloc
        h = C.c_void_p()
        rc = lib.orc_mesh_create(self.E, self.N, _p(xyz), _p(glo), _p(bnd),
                                 None if kk is None else _p(kk), float(helm_h), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_mesh_create failed with code {rc}")
        self._h = h
        self.helm_h = float(helm_h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_mesh_destroy(h)
            self._h = None

    # --- data accessors ---------------------------------------------------
    def _get(self, what: int, size: int) -> np.ndarray:
        out = np.zeros(size)
        _lib.orc_mesh_get(self._h, what, _p(out))
        return out

    @property
    def G(self):
        return self._get(0, 6 * self.nloc).reshape(self.E, 6, self.n ** 3)

    @property
    def B(self):
        return self._get(1, self.nloc)

    @property
    def mult(self):
        return self._get(2, self.nloc)

    @property
    def c(self):
        return self._get(3, self.nloc)

    @property
    def dinv(self):
        return self._get(4, self.nloc)

    @property
    def D(self):
        return self._get(5, self.n * self.n).reshape(self.n, self.n)

    @property
    def mask(self):
        return self._get(6, self.nloc).astype(bool)

    @property
    def ngroups(self) -> int:
        return int(_lib.orc_mesh_ngroups(self._h))

    @property
    def mindet(self) -> float:
        return float(_lib.orc_mesh_mindet(self._h))

    # --- operators ---------------------------------------------------------
    def _unary(self, fn, u):
        u = _f64(u).reshape(-1)
        assert u.size == self.nloc
        w = np.zeros(self.nloc)
        fn(self._h, _p(u), _p(w))
        return w

    def ax_local(self, u):
        return self._unary(_lib.orc_ax_local, u)

    def apply(self, u):
        return self._unary(_lib.orc_apply, u)

    def rhs(self, f):
        return self._unary(_lib.orc_rhs, f)

    def gs(self, v):
        v = _f64(v).reshape(-1).copy()
        _lib.orc_gs(self._h, _p(v))
        return v

    def mask_apply(self, v):
        v = _f64(v).reshape(-1).copy()
        _lib.orc_mask(self._h, _p(v))
        return v

    def diag(self):
        d = np.zeros(self.nloc)
        _lib.orc_diag(self._h, _p(d))
        return d

    def dot(self, a, b) -> float:
        a = _f64(a).reshape(-1)
        b = _f64(b).reshape(-1)
        return float(_lib.orc_dot(self._h, _p(a), _p(b)))

    def dot_c_f32(self, a, b, dot2: bool) -> np.float32:
        """(a, b)_c in FP32: terms (fl(a_i c_i), b_i), Dot2 or recursive sum."""
        a, b = _f32(a), _f32(b)
        return np.float32(_lib.orc_dot_c_f32(self._h, 1 if dot2 else 0, _p(a), _p(b)))

    def gs_f32(self, v, acc64: bool, pairwise: bool, erank=None) -> np.ndarray:
        """QQ^T on an FP32 vector: FP64 or FP32 sums, one order per group or
        the pairwise order between ranks (erank [E] or None: every element
        a rank of its own); see orc_gs_f32."""
        v = _f32(v).copy()
        er = None if erank is None else np.ascontiguousarray(erank, dtype=np.int32)
        rc = _lib.orc_gs_f32(self._h, _p(v), 1 if acc64 else 0, 1 if pairwise else 0,
                             None if er is None else _p(er))
        if rc != 0:
            raise ValueError(f"orc_gs_f32 failed: {rc}")
        return v

    # --- solvers -----------------------------------------------------------
    def pcg(self, b, pc=PC_JACOBI, tol=1e-10, maxit=1000, x0=None, history=False, nn=None,
            mg=None):
        b = _f64(b).reshape(-1)
        x = np.zeros(self.nloc) if x0 is None else _f64(x0).reshape(-1).copy()
        hist = np.zeros(maxit + 1) if history else None
        st = _Stats()
        if mg is not None:
            pc, obj = PC_MG, mg._h
        else:
            obj = None if nn is None else nn._h
        rc = _lib.orc_pcg(self._h, pc, obj, _p(b), _p(x),
                          0 if x0 is None else 1, tol, maxit,
                          None if hist is None else _p(hist), C.byref(st))
        if rc != 0:
            raise RuntimeError(rc)
        s = _stats(st)
        if history:
            return x, s, hist[: s.iterations + 1]
        return x, s

    def fcg(self, b, nn=None, pc=None, tol=1e-10, maxit=1000, history=False):
        b = _f64(b).reshape(-1)
        x = np.zeros(self.nloc)
        hist = np.zeros(maxit + 1) if history else None
        st = _Stats()
        if pc is None:
            pc = PC_NN if nn is not None else PC_JACOBI
        rc = _lib.orc_fcg(self._h, pc, None if nn is None else nn._h, _p(b), _p(x), tol,
                          maxit, None if hist is None else _p(hist), C.byref(st))
        if rc != 0:
            raise RuntimeError(rc)
        s = _stats(st)
        if history:
            return x, s, hist[: s.iterations + 1]
        return x, s

    def ir(self, b, tol=1e-10, tau_in=1e-4, max_outer=10, inner_maxit=10000, pc=PC_JACOBI):
        b = _f64(b).reshape(-1)
        x = np.zeros(self.nloc)
        outer = np.zeros(max_outer + 1)
        st = _Stats()
        rc = _lib.orc_ir(self._h, pc, _p(b), _p(x), tol, tau_in, max_outer, inner_maxit,
                         _p(outer), C.byref(st))
        if rc != 0:
            raise RuntimeError(rc)
        s = _stats(st)
        return x, s, outer[: s.outer + 1]


class MG:
    """Oracle copy of the two-level Schwarz / multigrid preconditioner of a
    Dirichlet box mesh of ne^3 elements (lexicographic)."""

    def __init__(self, mesh: Mesh, ne: int, xyz, kcoef=None, coarsest_max: int = 512):
        _load()
        self.mesh = mesh
        self._xyz = _f64(xyz).reshape(-1)
        self._k = None if kcoef is None else _f64(kcoef).reshape(-1)
        h = C.c_void_p()
        rc = _lib.orc_mg_create(mesh._h, ne, _p(self._xyz),
                                None if self._k is None else _p(self._k), coarsest_max,
                                C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_mg_create failed: {rc}")
        self._h = h
        self.ne = ne
        self.nlev = _lib.orc_mg_nlev(h)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.orc_mg_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _local_op(self, fn, r):
        r = _f64(r).reshape(-1)
        z = np.zeros(self.mesh.nloc)
        getattr(_lib, fn)(self.mesh._h, self._h, _p(r), _p(z))
        return z

    def apply(self, r):
        return self._local_op("orc_mg_apply", r)

    def schwarz_local(self, r):
        return self._local_op("orc_mg_schwarz_local", r)

    def level_nu(self, l: int) -> int:
        return _lib.orc_mg_level_nu(self._h, l)

    def level_omega(self, l: int) -> float:
        return _lib.orc_mg_level_omega(self._h, l)

    def level_dense(self, l: int) -> np.ndarray:
        nn = self.level_nu(l) ** 3
        A = np.zeros((nn, nn))
        _lib.orc_mg_level_dense(self._h, l, _p(A))
        return A

    def restrict(self, r):
        r = _f64(r).reshape(-1)
        rc = np.zeros(self.level_nu(0) ** 3)
        _lib.orc_mg_restrict(self.mesh._h, self._h, _p(r), _p(rc))
        return rc

    def prolong_add(self, zc, z):
        zc = _f64(zc).reshape(-1)
        z = _f64(z).reshape(-1).copy()
        _lib.orc_mg_prolong_add(self.mesh._h, self._h, _p(zc), _p(z))
        return z

    def vcycle(self, b):
        b = _f64(b).reshape(-1)
        x = np.zeros_like(b)
        _lib.orc_mg_vcycle(self._h, _p(b), _p(x))
        return x

    def eig(self, e: int, d: int):
        n = self.mesh.n
        S = np.zeros((n, n))
        lam = np.zeros(n)
        _lib.orc_mg_eig(self._h, e, d, _p(S), _p(lam))
        return S, lam


def _stats(st: _Stats) -> SolveStats:
    return SolveStats(st.iterations, st.reason, st.outer, st.fallback,
                      st.rel_res_recursive, st.rel_res_true)


class NN:
    """Oracle copy of the per-element convolutional correction (FP64)."""

    def __init__(self, W1, W2, cin: int = 2):
        lib = _load()
        W1 = _f64(W1)
        W2 = _f64(W2)
        self.ch = W2.size // 27
        self.cin = cin
        assert W1.size == self.ch * cin * 27
        h = C.c_void_p()
        rc = lib.orc_nn_create(cin, self.ch, _p(W1), _p(W2), C.byref(h))
        if rc != 0:
            raise ValueError(rc)
        self._h = h
        self.W1 = W1.reshape(self.ch, cin, 27).copy()
        self.W2 = W2.reshape(self.ch, 27).copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_nn_destroy(h)
            self._h = None

    def set(self, W1, W2):
        W1 = _f64(W1)
        W2 = _f64(W2)
        _lib.orc_nn_set(self._h, _p(W1), _p(W2))
        self.W1 = W1.reshape(self.ch, self.cin, 27).copy()
        self.W2 = W2.reshape(self.ch, 27).copy()

    def local(self, mesh: Mesh, r):
        r = _f64(r).reshape(-1)
        zL = np.zeros(mesh.nloc)
        y = np.zeros(mesh.nloc)
        _lib.orc_nn_local(mesh._h, self._h, _p(r), _p(zL), _p(y))
        return zL, y

    def apply(self, mesh: Mesh, r):
        r = _f64(r).reshape(-1)
        z = np.zeros(mesh.nloc)
        _lib.orc_nn_apply(mesh._h, self._h, _p(r), _p(z))
        return z

    def loss_grad(self, mesh: Mesh, R, Eerr):
        R = _f64(R)
        Eerr = _f64(Eerr)
        ns = R.size // mesh.nloc
        assert R.size == ns * mesh.nloc and Eerr.size == R.size
        loss = np.zeros(1)
        g1 = np.zeros(self.ch * self.cin * 27)
        g2 = np.zeros(self.ch * 27)
        rc = _lib.orc_nn_loss_grad(mesh._h, self._h, ns, _p(R), _p(Eerr), _p(loss), _p(g1),
                                   _p(g2))
        if rc != 0:
            raise RuntimeError(rc)
        return float(loss[0]), g1.reshape(self.ch, self.cin, 27), g2.reshape(self.ch, 27)


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (theta, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam(theta.size, _p(theta), _p(g), _p(m), _p(v), t, lr, b1, b2, eps)
