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
    assert L.mxsem_mesh_create(None, None, None) == mx.EINVAL
    assert L.mxsem_solve(None, None, None, None, None) == mx.EINVAL
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
