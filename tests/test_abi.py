"""The C-ABI library loads and exports every symbol include/mxsem.h declares;
host-only entry points (no GPU needed) behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mxsem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mxsem_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def mx():
    from paper_2503_02134_amd import mxsem
    if not os.path.exists(mxsem.LIB_PATH):
        from paper_2503_02134_amd import build
        build.build()
    mxsem.lib()
    return mxsem


def test_every_declared_symbol_is_exported(mx):
    names = _declared()
    assert len(names) >= 30
    L = mx.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version(mx):
    L = mx.lib()
    assert L.mxsem_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.mxsem_status_str(code)
    assert L.mxsem_status_str(-99) == b"unknown status"


def test_library_gll_matches_oracle(mx, orc):
    """The library's reference element (own Newton iteration on
    L_{N+1} - L_{N-1}) agrees with the oracle's."""
    for N in range(1, 16):
        xl, wl = mx.mxsem_gll(N)
        xo, wo = orc.gll(N)
        np.testing.assert_allclose(xl, xo, atol=2e-15)
        np.testing.assert_allclose(wl, wo, rtol=2e-13)


def test_invalid_arguments_rejected(mx):
    L = mx.lib()
    xi = np.zeros(17)
    assert L.mxsem_gll(0, xi.ctypes.data, xi.ctypes.data) == mx.ENOTSUP
    assert L.mxsem_gll(16, xi.ctypes.data, xi.ctypes.data) == mx.ENOTSUP
    assert L.mxsem_gll(3, None, None) == mx.EINVAL
    assert L.mxsem_ctx_create(0, None, None) == mx.EINVAL
    assert L.mxsem_mesh_create(None, None, None, 0, None) == mx.EINVAL
    assert L.mxsem_solve(None, None, None, None, None) == mx.EINVAL
    assert L.mxsem_stream_copy(None, None, None, 16) == mx.EINVAL
    assert L.mxsem_stream_mix(None, None, 64, None, 16) == mx.EINVAL
    assert b"null" in L.mxsem_last_error()
    o = mx.solve_opts()
    assert o.tol == 1e-10 and o.graph_chunk >= 1 and o.inner_tol == 1e-4


def test_product_path_has_no_oracle_dependency():
    """Nothing in the package imports, links or names the oracle."""
    pkg = os.path.join(ROOT, "paper_2503_02134_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f
                assert "from oracle" not in txt, f


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library every call fails at once (no CPU path):
    a fresh interpreter whose library path points at a missing file."""
    import subprocess
    import sys
    code = (
        "from paper_2503_02134_amd import mxsem\n"
        f"mxsem.LIB_PATH = {str(tmp_path / 'libmxsem.so')!r}\n"
        "try:\n"
        "    mxsem.mxsem_gll(3)\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "else:\n"
        "    print('no error')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert "raised:" in out.stdout and "is not built" in out.stdout


def test_binding_constants_match_header():
    """Every enum value and integer #define of include/mxsem.h has the same
    value under the binding's name (the header name without MXSEM_)."""
    from paper_2503_02134_amd import mxsem
    src = open(os.path.join(ROOT, "include", "mxsem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {}
    for name, v in re.findall(r"\bMXSEM_([A-Z0-9_]+)\s*=\s*(-?\d+)", src):
        vals[name] = int(v)
    for name, v in re.findall(r"#define\s+MXSEM_([A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", src):
        vals[name] = int(v)
    assert len(vals) >= 35
    missing = [n for n in vals if not hasattr(mxsem, n)]
    assert missing == [], missing
    for n, v in vals.items():
        assert getattr(mxsem, n) == v, n


def test_binding_checks_vectors_before_any_launch(mx, monkeypatch):
    """Every device vector is checked (torch tensor, dtype of the call's
    precision, contiguous, number of entries, device) before the library is
    called, so a wrong vector raises instead of letting a kernel run past
    its end.  A mesh the binding knows of is faked here (no GPU): each bad
    vector raises, and a vector that passes every other check still raises
    because it is not on the device."""
    import torch
    fake = 0x1234
    monkeypatch.setitem(mx._mesh_shape, fake, mx._MeshShape(nloc=8, device=0))

    def boom(*a, **k):
        raise AssertionError("the library was called")

    class _NoLib:
        def __getattr__(self, name):
            return boom

    monkeypatch.setattr(mx, "lib", lambda: _NoLib())
    f64 = torch.zeros(8, dtype=torch.float64)
    f32 = torch.zeros(8, dtype=torch.float32)
    cases = [
        (TypeError, lambda: mx.mxsem_apply(fake, mx.F64, f64.numpy(), f64)),      # not a tensor
        (TypeError, lambda: mx.mxsem_apply(fake, mx.F64, f32, f64)),              # dtype vs io
        (TypeError, lambda: mx.mxsem_apply(fake, mx.F32, f64, f32)),
        (TypeError, lambda: mx.mxsem_apply(fake, mx.BF16G_F32, f64, f64)),
        (ValueError, lambda: mx.mxsem_apply(fake, mx.F64, torch.zeros(7, dtype=torch.float64), f64)),
        (ValueError, lambda: mx.mxsem_apply(fake, mx.F64, torch.zeros(16, dtype=torch.float64)[::2], f64)),
        (ValueError, lambda: mx.mxsem_apply(fake, mx.F64, f64, f64)),             # CPU tensors
        (TypeError, lambda: mx.mxsem_gather_scatter(fake, mx.F32, mx.F64, f64)),
        (ValueError, lambda: mx.mxsem_gather_scatter(fake, mx.F64, mx.F64, torch.zeros(9, dtype=torch.float64))),
        (TypeError, lambda: mx.mxsem_dot(fake, mx.F32, f64, f32, torch.zeros(1, dtype=torch.float64))),
        (TypeError, lambda: mx._scalar64(fake, torch.zeros(1, dtype=torch.float32), "out")),
        (ValueError, lambda: mx._scalar64(fake, torch.zeros(0, dtype=torch.float64), "out")),
        (TypeError, lambda: mx.mxsem_precond(fake, mx.PC_JACOBI, mx.F64, f32, f32)),
        (TypeError, lambda: mx.mxsem_mass_rhs(fake, f32, f64)),
        (TypeError, lambda: mx.mxsem_solve(fake, _opts(mx), f32, f64)),
        (ValueError, lambda: mx.mxsem_solve(fake, _opts(mx), torch.zeros(4, dtype=torch.float64), f64)),
        (ValueError, lambda: mx.mxsem_nn_make_pair(fake, f64, f64, f64, torch.zeros(3, dtype=torch.float32), f32)),
        (ValueError, lambda: mx._shape(0x999)),                                   # unknown mesh
    ]
    for exc, call in cases:
        with pytest.raises(exc):
            call()
    # a history shorter than max_iter + 1 is refused
    o = _opts(mx)
    o.max_iter = 10
    o._history = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="history"):
        mx._check_history(fake, o)
    o._history = torch.zeros(11, dtype=torch.float32)
    with pytest.raises(TypeError, match="history"):
        mx._check_history(fake, o)
    # networks: r and e hold nsamp vectors, the gradient every parameter
    monkeypatch.setitem(mx._nn_mesh, 0x77, fake)
    loss = torch.zeros(1, dtype=torch.float64)
    with pytest.raises(ValueError):
        mx.mxsem_nn_loss_grad(0x77, torch.zeros(8, dtype=torch.float32), f32, 2, loss, None)
    with pytest.raises(ValueError):
        mx.mxsem_nn_loss_grad(0x77, torch.zeros(16, dtype=torch.float32),
                              torch.zeros(16, dtype=torch.float32), 2, loss,
                              torch.zeros(mx.NN_PARAMS - 1, dtype=torch.float32))
    with pytest.raises(TypeError):
        mx.mxsem_nn_forward(0x77, f64, f32)


def _opts(mx):
    """Solve options built without the library (the fake above has none)."""
    o = mx.mxsem_solve_opts()
    o.max_iter = 100
    o._history = None
    o.history = None
    return o


def _small_desc(mx, ne=2, N=3, views=None):
    from paper_2503_02134_amd import workloads as W
    xi, _ = mx.mxsem_gll(N)
    bm = W.box_mesh(ne, N, xi)
    v = (mx.VIEW_F64 | mx.VIEW_F32 | mx.VIEW_BF16) if views is None else views
    return bm, mx._mesh_desc(bm.E, N, bm.xyz, bm.glo, bm.bnd, None, 0.0, v)


def test_mesh_workspace_is_sized_and_checked_on_the_host(mx):
    """The library allocates no device memory: a mesh lives in a caller
    workspace whose size mxsem_mesh_workspace_bytes reports (host work
    only).  mesh_create refuses a null, misaligned or undersized workspace
    with MXSEM_EINVAL before it touches the device (no context needed to
    see it), and only then asks for the context."""
    L = mx.lib()
    bm, (d, keep) = _small_desc(mx)
    nb = C.c_size_t()
    assert L.mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb)) == mx.OK
    full = nb.value
    # FP64 operator, solver vectors and both FP32 precisions: well over the
    # 8-byte vectors alone, and a multiple of 256 bytes
    assert full % 256 == 0 and full > 20 * 8 * bm.nloc
    bm64, (d64, keep64) = _small_desc(mx, views=mx.VIEW_F64)
    assert L.mxsem_mesh_workspace_bytes(C.byref(d64), C.byref(nb)) == mx.OK
    assert nb.value < full
    fake = 1 << 40  # never dereferenced: every check below fails first
    h = C.c_void_p()
    for ptr, size in ((None, full), (fake + 8, full), (fake, full - 256), (fake, 0)):
        assert L.mxsem_mesh_create(None, C.byref(d), ptr, size, C.byref(h)) == mx.EINVAL
        assert b"workspace" in L.mxsem_last_error()
    assert L.mxsem_mesh_create(None, C.byref(d), fake, full, C.byref(h)) == mx.EINVAL
    assert b"null context" in L.mxsem_last_error()
    # descriptor errors are the same in both calls
    d.N = 16
    assert L.mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb)) == mx.ENOTSUP
    assert L.mxsem_mesh_create(None, C.byref(d), fake, full, C.byref(h)) == mx.ENOTSUP


def test_autotune_workspace_bytes(mx):
    L = mx.lib()
    nb = C.c_size_t()
    assert L.mxsem_autotune_workspace_bytes(7, 64, mx.F32, C.byref(nb)) == mx.OK
    nloc = 64 * 512
    assert nb.value >= (4 + 4 + 24) * nloc  # u, w and six FP32 factors per node
    assert L.mxsem_autotune_workspace_bytes(16, 64, mx.F32, C.byref(nb)) == mx.ENOTSUP
    assert L.mxsem_autotune_workspace_bytes(7, 0, mx.F32, C.byref(nb)) == mx.EINVAL


def test_multigrid_view_is_sized_and_checked_on_the_host(mx):
    """MXSEM_VIEW_MG adds the multigrid blocks to the mesh workspace, and a
    mesh that is not a Dirichlet box of lexicographic elements is refused
    with MXSEM_ENOTSUP by the sizing call already."""
    L = mx.lib()
    bm, (d, keep) = _small_desc(mx, ne=4, N=3)
    nb0, nb1 = C.c_size_t(), C.c_size_t()
    assert L.mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb0)) == mx.OK
    d.views |= mx.VIEW_MG
    assert L.mxsem_mesh_workspace_bytes(C.byref(d), C.byref(nb1)) == mx.OK
    # eigenvector matrices (3 n^2 per element, FP64 and FP32), lattice stencils
    assert nb1.value - nb0.value >= bm.E * 3 * 16 * 12
    glo = np.ascontiguousarray(bm.glo.reshape(bm.E, -1)[::-1])
    bm2, (d2, keep2) = _small_desc(mx, ne=4, N=3)
    d2.glo = glo.ctypes.data
    d2.views |= mx.VIEW_MG
    assert L.mxsem_mesh_workspace_bytes(C.byref(d2), C.byref(nb1)) == mx.ENOTSUP
    assert b"lattice" in L.mxsem_last_error()
    d2.views = 16
    assert L.mxsem_mesh_workspace_bytes(C.byref(d2), C.byref(nb1)) == mx.EINVAL


def test_tuning_struct_and_mapping_checks(mx):
    """mxsem_tuning carries a tile and a thread mapping per order; a mapping
    outside 0..2, or two columns where the order has no such kernel, is
    refused before anything runs (a null mesh is refused first)."""
    import ctypes as C
    assert C.sizeof(mx.mxsem_tuning) == 2 * 16 * C.sizeof(C.c_int)
    t = mx.mxsem_tuning()
    assert mx.lib().mxsem_mesh_set_tuning(None, C.byref(t)) == mx.EINVAL
