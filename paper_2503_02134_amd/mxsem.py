"""ctypes binding of libmxsem.so (the C ABI in include/mxsem.h).

Argument marshalling only: every numerical step runs in the HIP kernels of
the library.  Device vectors are torch tensors on the context's device;
their data pointers are passed through unchanged.  If the library is not
built or cannot be loaded, every call raises: there is no CPU fallback.

torch is imported before the library is loaded so that the library binds
to the HIP runtime torch already holds (one runtime per process).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (must precede loading the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmxsem.so")

# status codes
OK, EINVAL, ENOTSUP, EHIP, EBREAKDOWN, EINTERNAL, ENOMEM, EMESH = 0, -1, -2, -3, -4, -5, -6, -7
# precisions
F64, F32, BF16G_F32 = 0, 1, 2
# preconditioners
PC_IDENTITY, PC_JACOBI, PC_LEARNED, PC_MG = 0, 1, 2, 3
# modes
MODE_FP64, MODE_MIXED, MODE_MIXED_IR, MODE_MIXED_IR_BF16G, MODE_FP32_ALL = 0, 1, 2, 3, 4
MODE_MIXED_IR_BF16P = 5
METHOD_PCG, METHOD_FCG = 0, 1
CONVERGED, MAX_ITER, STAGNATED, BREAKDOWN = 1, 2, 3, 4
LOCAL_ONLY, MASK, GS_PAIRWISE = 1, 2, 4
# dot accumulation of the FP32 loop, and gather-scatter order
DOT_DEFAULT, DOT_F64, DOT_F32, DOT_DOT2 = 0, 1, 2, 3
GS_ORDER_ONE, GS_ORDER_PAIRWISE = 0, 1
VIEW_F64, VIEW_F32, VIEW_BF16, VIEW_MG = 1, 2, 4, 8

MODE_NAMES = {MODE_FP64: "fp64", MODE_MIXED: "mixed", MODE_MIXED_IR: "mixed_ir",
              MODE_MIXED_IR_BF16G: "mixed_ir_bf16g", MODE_FP32_ALL: "fp32_all",
              MODE_MIXED_IR_BF16P: "mixed_ir_bf16p"}


class MxsemError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class mxsem_mesh_desc(C.Structure):
    _fields_ = [("E", C.c_int), ("N", C.c_int), ("xyz", C.c_void_p), ("glo", C.c_void_p),
                ("bnd", C.c_void_p), ("kcoef", C.c_void_p), ("helm_h", C.c_double),
                ("views", C.c_uint)]


class mxsem_solve_opts(C.Structure):
    _fields_ = [("method", C.c_int), ("pc", C.c_int), ("mode", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("inner_tol", C.c_double), ("max_outer", C.c_int),
                ("graph_chunk", C.c_int), ("x0_given", C.c_int), ("history", C.c_void_p),
                ("dot", C.c_int), ("gs_order", C.c_int)]


class mxsem_solve_stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer", C.c_int), ("reason", C.c_int),
                ("fallback_used", C.c_int), ("rel_res", C.c_double),
                ("rel_res_recursive", C.c_double), ("ms", C.c_double), ("ax_ms", C.c_double),
                ("ax_samples", C.c_int), ("pad_", C.c_int)]


class mxsem_tuning(C.Structure):
    _fields_ = [("epb", C.c_int * 16), ("cols", C.c_int * 16)]


class mxsem_nn_desc(C.Structure):
    _fields_ = [("cin", C.c_int), ("ch", C.c_int), ("max_samples", C.c_int)]


class mxsem_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("step", C.c_int)]


_lib = None
vp = C.c_void_p
_SIGS = {
    "mxsem_ctx_create": [C.c_int, vp, C.POINTER(vp)],
    "mxsem_ctx_destroy": [vp],
    "mxsem_ctx_set_stream": [vp, vp],
    "mxsem_gll": [C.c_int, vp, vp],
    "mxsem_mesh_workspace_bytes": [C.POINTER(mxsem_mesh_desc), C.POINTER(C.c_size_t)],
    "mxsem_mesh_create": [vp, C.POINTER(mxsem_mesh_desc), vp, C.c_size_t, C.POINTER(vp)],
    "mxsem_mesh_destroy": [vp],
    "mxsem_mesh_info": [vp, vp, vp, vp, vp],
    "mxsem_mesh_get": [vp, C.c_int, vp],
    "mxsem_apply": [vp, C.c_int, vp, vp, C.c_uint],
    "mxsem_gather_scatter": [vp, C.c_int, C.c_int, vp, C.c_uint],
    "mxsem_dot": [vp, C.c_int, vp, vp, vp],
    "mxsem_dot_ex": [vp, C.c_int, C.c_int, vp, vp, vp],
    "mxsem_mesh_set_ranks": [vp, vp],
    "mxsem_precond": [vp, C.c_int, C.c_int, vp, vp],
    "mxsem_mass_rhs": [vp, vp, vp],
    "mxsem_solve": [vp, C.POINTER(mxsem_solve_opts), vp, vp, C.POINTER(mxsem_solve_stats)],
    "mxsem_batch_workspace_bytes": [vp, C.c_int, vp, C.c_char_p, C.POINTER(C.c_size_t)],
    "mxsem_batch_create": [vp, C.c_int, vp, C.c_char_p, vp, C.c_size_t, C.POINTER(vp)],
    "mxsem_batch_destroy": [vp],
    "mxsem_batch_solve": [vp, C.POINTER(mxsem_solve_opts), vp, vp, vp],
    "mxsem_autotune_workspace_bytes": [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)],
    "mxsem_autotune": [vp, C.c_int, C.c_int, C.c_int, vp, C.c_size_t, C.POINTER(mxsem_tuning)],
    "mxsem_mesh_set_tuning": [vp, C.POINTER(mxsem_tuning)],
    "mxsem_nn_workspace_bytes": [vp, C.POINTER(mxsem_nn_desc), C.POINTER(C.c_size_t)],
    "mxsem_nn_create": [vp, C.POINTER(mxsem_nn_desc), vp, C.c_size_t, C.POINTER(vp)],
    "mxsem_nn_destroy": [vp],
    "mxsem_nn_set_params": [vp, vp, vp],
    "mxsem_nn_get_params": [vp, vp, vp],
    "mxsem_nn_forward": [vp, vp, vp],
    "mxsem_nn_loss_grad": [vp, vp, vp, C.c_int, vp, vp],
    "mxsem_nn_adam_step": [vp, C.POINTER(mxsem_adam)],
    "mxsem_mesh_attach_nn": [vp, vp],
    "mxsem_nn_make_pair": [vp, vp, vp, vp, vp, vp],
    "mxsem_stream_copy": [vp, vp, vp, C.c_size_t],
    "mxsem_stream_mix": [vp, vp, C.c_size_t, vp, C.c_size_t],
    "mxsem_version": [],
}


def lib():
    """Load libmxsem.so (raises if it is not built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python paper_2503_02134_amd/build.py")
    L = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.mxsem_status_str.argtypes = [C.c_int]
    L.mxsem_status_str.restype = C.c_char_p
    L.mxsem_last_error.argtypes = []
    L.mxsem_last_error.restype = C.c_char_p
    L.mxsem_solve_opts_default.argtypes = [C.POINTER(mxsem_solve_opts)]
    L.mxsem_solve_opts_default.restype = None
    _lib = L
    return L


def _check(fn: str, rc: int):
    if rc != OK:
        msg = lib().mxsem_last_error().decode(errors="replace")
        raise MxsemError(fn, rc, msg)


def _ptr(t) -> int | None:
    """Address of a host buffer (numpy array or integer address)."""
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        raise TypeError("host buffers are numpy arrays; device vectors go through _vec")
    if isinstance(t, np.ndarray):
        if not t.flags.c_contiguous:
            raise ValueError("host arrays must be C-contiguous")
        return t.ctypes.data
    return int(t)


# What the binding knows of each live handle, so that every device vector is
# checked before a call could make a kernel read or write past its end:
# meshes -> (local entries, device), networks -> mesh, batches -> meshes.
@dataclass
class _MeshShape:
    nloc: int
    device: int


_ctx_device: dict = {}
_mesh_shape: dict = {}
_nn_mesh: dict = {}
_batch_meshes: dict = {}
_batch_ws: dict = {}
NN_PARAMS = 32 * 2 * 27 + 32 * 27


def _key(h) -> int:
    return h.value if isinstance(h, C.c_void_p) else int(h or 0)


def _shape(mesh) -> _MeshShape:
    sh = _mesh_shape.get(_key(mesh))
    if sh is None:
        raise ValueError("unknown mesh handle (not created through this binding, or destroyed)")
    return sh


def _io_dtype(io: int):
    if io == F64:
        return torch.float64
    if io in (F32, BF16G_F32):
        return torch.float32
    raise ValueError(f"unknown precision {io}")


def _vec(t, dtype, n: int, device: int, what: str, at_least: bool = False) -> int:
    """Data pointer of a device vector after checking, in this order, that it
    is a torch tensor of the given dtype, contiguous, with n entries (at
    least n with at_least), on the given device; raises otherwise, before
    anything is launched."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise TypeError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if (t.numel() < n) if at_least else (t.numel() != n):
        raise ValueError(f"{what}: {t.numel()} entries, expected {'at least ' if at_least else ''}{n}")
    if t.device.type != "cuda" or (t.device.index or 0) != device:
        raise ValueError(f"{what}: tensor on {t.device}, expected cuda:{device}")
    return t.data_ptr()


# ---------------------------------------------------------------- C ABI, one to one
def mxsem_ctx_create(device: int = 0, stream=None):
    h = vp()
    s = torch.cuda.current_stream(device).cuda_stream if stream is None else stream
    _check("mxsem_ctx_create", lib().mxsem_ctx_create(device, s, C.byref(h)))
    _ctx_device[_key(h)] = int(device)
    return h


def mxsem_ctx_destroy(ctx):
    _check("mxsem_ctx_destroy", lib().mxsem_ctx_destroy(ctx))
    _ctx_device.pop(_key(ctx), None)


def mxsem_gll(N: int):
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    _check("mxsem_gll", lib().mxsem_gll(N, xi.ctypes.data, w.ctypes.data))
    return xi, w


def _workspace(nbytes: int, device: int) -> torch.Tensor:
    """Caller-owned device workspace (torch's allocator; 256-byte aligned)."""
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=torch.device("cuda", device))
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return ws


def _mesh_desc(E, N, xyz, glo, bnd, kcoef, helm_h, views):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    glo = np.ascontiguousarray(glo, dtype=np.int64)
    bnd = np.ascontiguousarray(bnd, dtype=np.uint8)
    kk = None if kcoef is None else np.ascontiguousarray(kcoef, dtype=np.float64)
    n3 = (N + 1) ** 3
    if not (xyz.size == 3 * E * n3 and glo.size == E * n3 and bnd.size == E * n3
            and (kk is None or kk.size == E * n3)):
        raise ValueError("mesh arrays do not match E and N")
    d = mxsem_mesh_desc(E, N, xyz.ctypes.data, glo.ctypes.data, bnd.ctypes.data,
                        None if kk is None else kk.ctypes.data, float(helm_h), views)
    return d, (xyz, glo, bnd, kk)  # the arrays must outlive the call


def mxsem_mesh_workspace_bytes(E, N, xyz, glo, bnd, kcoef=None, helm_h=0.0,
                               views=VIEW_F64 | VIEW_F32 | VIEW_BF16) -> int:
    d, _keep = _mesh_desc(E, N, xyz, glo, bnd, kcoef, helm_h, views)
    nb = C.c_size_t()
    _check("mxsem_mesh_workspace_bytes", lib().mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb)))
    return nb.value


def mxsem_mesh_create(ctx, E, N, xyz, glo, bnd, kcoef=None, helm_h=0.0,
                      views=VIEW_F64 | VIEW_F32 | VIEW_BF16, workspace=None):
    """Returns (handle, workspace tensor); the tensor must outlive the mesh.
    With workspace=None one of the size mxsem_mesh_workspace_bytes reports is
    allocated here."""
    d, _keep = _mesh_desc(E, N, xyz, glo, bnd, kcoef, helm_h, views)
    dev = _ctx_device.get(_key(ctx), 0)
    if workspace is None:
        nb = C.c_size_t()
        _check("mxsem_mesh_workspace_bytes",
               lib().mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb)))
        workspace = _workspace(nb.value, dev)
    pw = _vec(workspace, torch.uint8, 0, dev, "mesh_create: workspace", at_least=True)
    h = vp()
    _check("mxsem_mesh_create", lib().mxsem_mesh_create(ctx, C.byref(d), pw, workspace.numel(),
                                                         C.byref(h)))
    _mesh_shape[_key(h)] = _MeshShape(E * (N + 1) ** 3, dev)
    return h, workspace


def mxsem_mesh_destroy(mesh):
    _check("mxsem_mesh_destroy", lib().mxsem_mesh_destroy(mesh))
    _mesh_shape.pop(_key(mesh), None)


def mxsem_mesh_info(mesh):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    d = C.c_double()
    _check("mxsem_mesh_info", lib().mxsem_mesh_info(mesh, C.byref(a), C.byref(b), C.byref(c),
                                                     C.byref(d)))
    return a.value, b.value, c.value, d.value


def mxsem_mesh_get(mesh, what: int, size: int) -> np.ndarray:
    out = np.zeros(size)
    _check("mxsem_mesh_get", lib().mxsem_mesh_get(mesh, what, out.ctypes.data))
    return out


def _local(mesh, io, t, what):
    sh = _shape(mesh)
    return _vec(t, _io_dtype(io), sh.nloc, sh.device, what)


def _scalar64(mesh, t, what):
    return _vec(t, torch.float64, 1, _shape(mesh).device, what, at_least=True)


def mxsem_apply(mesh, prec, u, w, flags=0):
    pu, pw = _local(mesh, prec, u, "apply: u"), _local(mesh, prec, w, "apply: w")
    _check("mxsem_apply", lib().mxsem_apply(mesh, prec, pu, pw, flags))


def mxsem_gather_scatter(mesh, io, acc, v, flags=0):
    pv = _local(mesh, io, v, "gather_scatter: v")
    _check("mxsem_gather_scatter", lib().mxsem_gather_scatter(mesh, io, acc, pv, flags))


def mxsem_dot(mesh, io, a, b, out_dev):
    pa, pb = _local(mesh, io, a, "dot: a"), _local(mesh, io, b, "dot: b")
    po = _scalar64(mesh, out_dev, "dot: out")
    _check("mxsem_dot", lib().mxsem_dot(mesh, io, pa, pb, po))


def mxsem_dot_ex(mesh, io, acc, a, b, out_dev):
    pa, pb = _local(mesh, io, a, "dot_ex: a"), _local(mesh, io, b, "dot_ex: b")
    po = _scalar64(mesh, out_dev, "dot_ex: out")
    _check("mxsem_dot_ex", lib().mxsem_dot_ex(mesh, io, acc, pa, pb, po))


def mxsem_mesh_set_ranks(mesh, ranks):
    """ranks: int32 array [E] (host) or None (every element a rank of its own)."""
    if ranks is None:
        _check("mxsem_mesh_set_ranks", lib().mxsem_mesh_set_ranks(mesh, None))
        return
    import numpy as np
    arr = np.ascontiguousarray(ranks, dtype=np.int32)
    _check("mxsem_mesh_set_ranks", lib().mxsem_mesh_set_ranks(mesh, arr.ctypes.data_as(C.c_void_p)))


def mxsem_precond(mesh, pc, io, r, z):
    pr, pz = _local(mesh, io, r, "precond: r"), _local(mesh, io, z, "precond: z")
    _check("mxsem_precond", lib().mxsem_precond(mesh, pc, io, pr, pz))


def mxsem_mass_rhs(mesh, f, b):
    pf, pb = _local(mesh, F64, f, "mass_rhs: f"), _local(mesh, F64, b, "mass_rhs: b")
    _check("mxsem_mass_rhs", lib().mxsem_mass_rhs(mesh, pf, pb))


def solve_opts(**kw) -> mxsem_solve_opts:
    """Options with the library's defaults; history is a device FP64 tensor
    (checked against the mesh and max_iter when the solve is called)."""
    o = mxsem_solve_opts()
    lib().mxsem_solve_opts_default(C.byref(o))
    hist = kw.pop("history", None)
    for k, v in kw.items():
        setattr(o, k, v)
    o._history = hist
    o.history = None if hist is None else hist.data_ptr()
    return o


def _check_history(mesh, opts):
    hist = getattr(opts, "_history", None)
    if hist is not None:
        _vec(hist, torch.float64, opts.max_iter + 1, _shape(mesh).device, "solve: history",
             at_least=True)
    elif opts.history:
        raise ValueError("solve: pass the history as a tensor through solve_opts")


def mxsem_solve(mesh, opts: mxsem_solve_opts, b, x) -> mxsem_solve_stats:
    pb, px = _local(mesh, F64, b, "solve: b"), _local(mesh, F64, x, "solve: x")
    _check_history(mesh, opts)
    st = mxsem_solve_stats()
    rc = lib().mxsem_solve(mesh, C.byref(opts), pb, px, C.byref(st))
    if rc == EBREAKDOWN:
        return st
    _check("mxsem_solve", rc)
    return st


def mxsem_batch_create(ctx, meshes, tune_cache: str | None = None):
    """Returns the handle; the batch's workspace tensor is held here until
    mxsem_batch_destroy."""
    arr = (vp * len(meshes))(*[m.value if isinstance(m, vp) else m for m in meshes])
    tc = None if tune_cache is None else tune_cache.encode()
    nb = C.c_size_t()
    _check("mxsem_batch_workspace_bytes", lib().mxsem_batch_workspace_bytes(
        ctx, len(meshes), C.cast(arr, vp), tc, C.byref(nb)))
    ws = _workspace(nb.value, _ctx_device.get(_key(ctx), 0))
    h = vp()
    _check("mxsem_batch_create", lib().mxsem_batch_create(
        ctx, len(meshes), C.cast(arr, vp), tc, ws.data_ptr(), ws.numel(), C.byref(h)))
    _batch_meshes[_key(h)] = [_key(m) for m in meshes]
    _batch_ws[_key(h)] = ws
    return h


def mxsem_batch_destroy(batch):
    _check("mxsem_batch_destroy", lib().mxsem_batch_destroy(batch))
    _batch_meshes.pop(_key(batch), None)
    _batch_ws.pop(_key(batch), None)


def mxsem_batch_solve(batch, opts, bs, xs):
    ms = _batch_meshes.get(_key(batch))
    if ms is None:
        raise ValueError("unknown batch handle")
    P = len(ms)
    if len(bs) != P or len(xs) != P:
        raise ValueError(f"batch_solve: {P} problems, got {len(bs)} b and {len(xs)} x")
    if opts.history or getattr(opts, "_history", None) is not None:
        raise ValueError("batch_solve: no residual history for batches")
    barr = (vp * P)(*[_local(m, F64, b, f"batch_solve: b[{p}]") for p, (m, b) in enumerate(zip(ms, bs))])
    xarr = (vp * P)(*[_local(m, F64, x, f"batch_solve: x[{p}]") for p, (m, x) in enumerate(zip(ms, xs))])
    st = (mxsem_solve_stats * P)()
    rc = lib().mxsem_batch_solve(batch, C.byref(opts), C.cast(barr, vp), C.cast(xarr, vp),
                                 C.cast(st, vp))
    if rc != EBREAKDOWN:
        _check("mxsem_batch_solve", rc)
    return list(st)


def mxsem_autotune(ctx, N, E, prec) -> tuple:
    """(elements per workgroup, thread mapping) of the fastest operator
    kernel for (N, E, prec); mapping 0 means the order has one mapping."""
    nb = C.c_size_t()
    _check("mxsem_autotune_workspace_bytes",
           lib().mxsem_autotune_workspace_bytes(N, E, prec, C.byref(nb)))
    ws = _workspace(nb.value, _ctx_device.get(_key(ctx), 0))
    t = mxsem_tuning()
    _check("mxsem_autotune", lib().mxsem_autotune(ctx, N, E, prec, ws.data_ptr(), ws.numel(),
                                                   C.byref(t)))
    del ws
    return t.epb[N], t.cols[N]


def mxsem_mesh_set_tuning(mesh, epb_by_N: dict, cols_by_N: dict | None = None):
    """Operator tile (elements per workgroup) and, optionally, thread mapping
    (1: one column per thread, 2: two; 0: the default) per order N."""
    t = mxsem_tuning()
    for N, e in epb_by_N.items():
        t.epb[N] = e
    for N, c in (cols_by_N or {}).items():
        t.cols[N] = c
    _check("mxsem_mesh_set_tuning", lib().mxsem_mesh_set_tuning(mesh, C.byref(t)))


def mxsem_nn_create(mesh, ch=32, cin=2, max_samples=16):
    """Returns (handle, workspace tensor); the tensor must outlive the network."""
    d = mxsem_nn_desc(cin, ch, max_samples)
    nb = C.c_size_t()
    _check("mxsem_nn_workspace_bytes", lib().mxsem_nn_workspace_bytes(mesh, C.byref(d), C.byref(nb)))
    ws = _workspace(nb.value, _shape(mesh).device)
    h = vp()
    _check("mxsem_nn_create", lib().mxsem_nn_create(mesh, C.byref(d), ws.data_ptr(), ws.numel(),
                                                     C.byref(h)))
    _nn_mesh[_key(h)] = _key(mesh)
    return h, ws


def mxsem_nn_destroy(nn):
    _check("mxsem_nn_destroy", lib().mxsem_nn_destroy(nn))
    _nn_mesh.pop(_key(nn), None)


def _nn_shape(nn) -> _MeshShape:
    m = _nn_mesh.get(_key(nn))
    if m is None:
        raise ValueError("unknown network handle")
    return _shape(m)


def mxsem_nn_set_params(nn, W1, W2):
    W1 = np.ascontiguousarray(W1, dtype=np.float32)
    W2 = np.ascontiguousarray(W2, dtype=np.float32)
    _check("mxsem_nn_set_params", lib().mxsem_nn_set_params(nn, W1.ctypes.data, W2.ctypes.data))


def mxsem_nn_get_params(nn, ch=32, cin=2):
    W1 = np.zeros((ch, cin, 27), dtype=np.float32)
    W2 = np.zeros((ch, 27), dtype=np.float32)
    _check("mxsem_nn_get_params", lib().mxsem_nn_get_params(nn, W1.ctypes.data, W2.ctypes.data))
    return W1, W2


def mxsem_nn_forward(nn, r, z):
    sh = _nn_shape(nn)
    pr = _vec(r, torch.float32, sh.nloc, sh.device, "nn_forward: r")
    pz = _vec(z, torch.float32, sh.nloc, sh.device, "nn_forward: z")
    _check("mxsem_nn_forward", lib().mxsem_nn_forward(nn, pr, pz))


def mxsem_nn_loss_grad(nn, r, e, nsamp, loss_dev, grad_dev):
    sh = _nn_shape(nn)
    if nsamp < 1:
        raise ValueError("nn_loss_grad: nsamp must be >= 1")
    pr = _vec(r, torch.float32, nsamp * sh.nloc, sh.device, "nn_loss_grad: r")
    pe = _vec(e, torch.float32, nsamp * sh.nloc, sh.device, "nn_loss_grad: e")
    pl = _vec(loss_dev, torch.float64, 1, sh.device, "nn_loss_grad: loss", at_least=True)
    pg = (None if grad_dev is None else
          _vec(grad_dev, torch.float32, NN_PARAMS, sh.device, "nn_loss_grad: grad", at_least=True))
    _check("mxsem_nn_loss_grad", lib().mxsem_nn_loss_grad(nn, pr, pe, nsamp, pl, pg))


def mxsem_nn_adam_step(nn, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
    a = mxsem_adam(lr, beta1, beta2, eps, step)
    _check("mxsem_nn_adam_step", lib().mxsem_nn_adam_step(nn, C.byref(a)))


def mxsem_mesh_attach_nn(mesh, nn):
    _check("mxsem_mesh_attach_nn", lib().mxsem_mesh_attach_nn(mesh, nn))


def mxsem_nn_make_pair(mesh, b, x, xstar, r_out, e_out):
    ps = [_local(mesh, F64, t, f"nn_make_pair: {nm}") for t, nm in ((b, "b"), (x, "x"), (xstar, "xstar"))]
    pr = _local(mesh, F32, r_out, "nn_make_pair: r_out")
    pe = _local(mesh, F32, e_out, "nn_make_pair: e_out")
    _check("mxsem_nn_make_pair", lib().mxsem_nn_make_pair(mesh, *ps, pr, pe))


def mxsem_stream_copy(ctx, src, dst):
    """dst = src (device tensors of equal byte size, a multiple of 16)."""
    dev = _ctx_device.get(_key(ctx), 0)
    n = src.numel() * src.element_size()
    ps = _vec(src, src.dtype, src.numel(), dev, "stream_copy: src")
    pd = _vec(dst, src.dtype, src.numel(), dev, "stream_copy: dst")
    _check("mxsem_stream_copy", lib().mxsem_stream_copy(ctx, ps, pd, n))


def mxsem_stream_mix(ctx, src, dst):
    """dst = src[0:n] + src[n:2n] + ... (FP32 device tensors, dst of n
    entries, src of k n with k = 1, 2, 4 or 8, n a multiple of 4)."""
    dev = _ctx_device.get(_key(ctx), 0)
    ps = _vec(src, torch.float32, src.numel(), dev, "stream_mix: src")
    pd = _vec(dst, torch.float32, dst.numel(), dev, "stream_mix: dst")
    _check("mxsem_stream_mix", lib().mxsem_stream_mix(ctx, ps, src.numel() * 4, pd, dst.numel() * 4))


# ---------------------------------------------------------------- convenience
@dataclass
class Stats:
    iterations: int
    outer: int
    reason: int
    fallback_used: int
    rel_res: float
    rel_res_recursive: float
    ms: float
    ax_ms: float
    ax_samples: int

    @staticmethod
    def of(st: mxsem_solve_stats) -> "Stats":
        return Stats(st.iterations, st.outer, st.reason, st.fallback_used, st.rel_res,
                     st.rel_res_recursive, st.ms, st.ax_ms, st.ax_samples)


_live_contexts: "weakref.WeakSet[Context]" = weakref.WeakSet()


class Context:
    """One device + the torch stream current at creation.  Closing it first
    closes every mesh / batch / network created from it."""

    def __init__(self, device: int = 0):
        self.device = device
        self.h = mxsem_ctx_create(device)
        self.children: list = []
        _live_contexts.add(self)

    def _adopt(self, obj):
        self.children.append(weakref.ref(obj))

    def close(self):
        if self.h is None:
            return
        for ref in reversed(self.children):
            obj = ref()
            if obj is not None:
                obj.close()
        self.children = []
        torch.cuda.synchronize(self.device)
        mxsem_ctx_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@atexit.register
def _close_all():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Mesh:
    """Device mesh built from host arrays (box-mesh generator output)."""

    def __init__(self, ctx: Context, E, N, xyz, glo, bnd, kcoef=None, helm_h=0.0,
                 views=VIEW_F64 | VIEW_F32 | VIEW_BF16):
        self.ctx = ctx
        self.E, self.N, self.n = int(E), int(N), int(N) + 1
        self.nloc = self.E * self.n ** 3
        self.h, self.ws = mxsem_mesh_create(ctx.h, E, N, xyz, glo, bnd, kcoef, helm_h, views)
        self.dev = torch.device("cuda", ctx.device)
        ctx._adopt(self)

    def close(self):
        if self.h is not None:
            mxsem_mesh_destroy(self.h)
            self.h = None
            self.ws = None  # the library no longer uses it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return mxsem_mesh_info(self.h)

    def get(self, what: int):
        size = {0: 6 * self.nloc, 5: self.n * self.n}.get(what, self.nloc)
        return mxsem_mesh_get(self.h, what, size)

    def vec(self, dtype=torch.float64):
        return torch.zeros(self.nloc, dtype=dtype, device=self.dev)

    def apply(self, u, prec=F64, local_only=False):
        w = torch.empty_like(u)
        mxsem_apply(self.h, prec, u, w, LOCAL_ONLY if local_only else 0)
        return w

    def gs(self, v, acc=F64, mask=False, pairwise=False):
        v = v.clone()
        io = F64 if v.dtype == torch.float64 else F32
        flags = (MASK if mask else 0) | (GS_PAIRWISE if pairwise else 0)
        mxsem_gather_scatter(self.h, io, acc, v, flags)
        return v

    def dot(self, a, b, acc=DOT_DEFAULT) -> float:
        out = torch.zeros(1, dtype=torch.float64, device=self.dev)
        io = F64 if a.dtype == torch.float64 else F32
        if acc == DOT_DEFAULT:
            mxsem_dot(self.h, io, a, b, out)
        else:
            mxsem_dot_ex(self.h, io, acc, a, b, out)
        return float(out.item())

    def set_ranks(self, ranks):
        mxsem_mesh_set_ranks(self.h, ranks)

    def precond(self, r, pc=PC_JACOBI):
        z = torch.empty_like(r)
        mxsem_precond(self.h, pc, F64 if r.dtype == torch.float64 else F32, r, z)
        return z

    def mass_rhs(self, f):
        b = torch.empty_like(f)
        mxsem_mass_rhs(self.h, f, b)
        return b

    def solve(self, b, x=None, **kw):
        if x is None:
            x = torch.zeros_like(b)
        st = mxsem_solve(self.h, solve_opts(**kw), b, x)
        return x, Stats.of(st)
