"""CPU checks of the C ABI: the library loads, exports every entry point that
include/lddmm.h declares, and rejects invalid configurations on the host
(no device call is made by any of these)."""
import ctypes
import os
import re

import pytest

from paper_2008_12820_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lddmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lddmm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_2008_12820_amd._lib as mod
    missing = [n for n in _declared() if not hasattr(mod, n) and n not in (
        "lddmm_status_string", "lddmm_last_error")]
    assert not missing, missing


@pytest.mark.parametrize("n,nt,reg,beta,leray", [
    ((7, 8, 8), 4, 1, 1e-2, 0),       # odd
    ((8, 8, 6), 4, 1, 1e-2, 0),       # too small
    ((14, 8, 8), 4, 1, 1e-2, 0),      # prime factor 7
    ((8, 8, 2048), 4, 1, 1e-2, 0),    # too large
    ((8, 8, 8), 0, 1, 1e-2, 0),       # nt
    ((8, 8, 8), 4, 3, 1e-2, 0),       # reg
    ((8, 8, 8), 4, 1, 0.0, 0),        # beta
    ((8, 8, 8), 4, 1, float("nan"), 0),
    ((8, 8, 8), 4, 1, 1e-2, 2),       # leray flag
])
def test_invalid_config_rejected(n, nt, reg, beta, leray):
    cfg = L.make_config(n, nt, reg, beta)
    cfg.leray = leray
    out = ctypes.c_size_t()
    st = L.lib().lddmm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out))
    assert st == L.EINVAL
    assert len(L.last_error()) > 0
    h = ctypes.c_void_p(1234)
    assert L.lib().lddmm_plan_create(ctypes.byref(cfg), None, ctypes.byref(h)) == L.EINVAL
    assert h.value is None


def test_workspace_model():
    """Workspace grows like (c + k*nt) fields: the state history, grad m and
    grad m at X per time step, plus a fixed set of fields and FFT scratch."""
    cfg = L.make_config((256, 256, 256), 4, 2, 5e-4)
    b4 = L.lddmm_workspace_bytes(cfg)
    cfg8 = L.make_config((256, 256, 256), 8, 2, 5e-4)
    b8 = L.lddmm_workspace_bytes(cfg8)
    field = 4 * 256 ** 3
    per_step = (b8 - b4) / 4 / field
    assert 8.5 < per_step < 9.5  # m_j, lam_j, 3 grad m_j, 3 grad m_j(X), source s_j
    assert b4 < 120 * field      # a few GB at 256^3: far below 288 GB


def test_null_pointers_and_status_strings():
    assert L.lib().lddmm_workspace_bytes(None, None) == L.EINVAL
    for s in range(7):
        assert len(L.status_string(s)) > 0
    assert L.lib().lddmm_set_images(None, None, None) == L.EINVAL
    assert L.lib().lddmm_num_kernels() > 10
    assert L.lddmm_kernel_name(0) == "r2c_x3"


def test_config_flags():
    """FD8, trilinear interpolation and transport-only are the known flag bits;
    any other bit is rejected."""
    out = ctypes.c_size_t()
    for flags, want in ((L.FLAG_FD8, L.OK), (L.FLAG_FD8 | L.FLAG_TRANSPORT_ONLY, L.OK),
                        (L.FLAG_LINEAR_IP | L.FLAG_FD8, L.OK), (8, L.EINVAL), (16 | L.FLAG_FD8, L.EINVAL)):
        cfg = L.make_config((16, 16, 16), 2, 2, 1e-2, flags=flags)
        assert L.lib().lddmm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == want, flags


def test_missing_library_fails_loudly():
    """No fallback: without liblddmm.so the binding raises instead of
    computing anything on the host."""
    import subprocess
    import sys
    code = ("import paper_2008_12820_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/liblddmm.so'\n"
            "L._lib = None\n"
            "try:\n"
            "    L.lib()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "else:\n"
            "    raise SystemExit('no error')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0, r.stderr
    assert "raised" in r.stdout and "missing" in r.stdout


def test_product_sources_never_use_the_oracle():
    """The oracle is test infrastructure: nothing in the package (Python
    binding or HIP sources) imports, loads or includes it."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2008_12820_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            if not f.endswith((".py", ".hip", ".hpp", ".h", ".c")):
                continue
            text = open(os.path.join(dirpath, f), encoding="utf-8").read()
            for bad in ("import oracle", "from oracle", "liboracle", "lddmm_oracle"):
                assert bad not in text, (f, bad)
