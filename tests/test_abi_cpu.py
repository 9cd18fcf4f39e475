"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/ori.h declares, and rejects bad arguments before
touching the device."""

import ctypes
import os
import re

import pytest

import paper_1602_04691_amd as ori
from paper_1602_04691_amd import build as ori_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ori.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ori_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ori.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each one, and exports it
    for n in names:
        assert hasattr(ori, n), n
        assert n in ori.__all__, n
    assert all(hasattr(ori, n) for n in ori.__all__)


def test_supported_lengths_match_header():
    text = open(HEADER).read()
    m = re.search(r"L >= 2n - 1 from\s*\*\s*\{([0-9,\s*]+)\}", text)
    listed = [int(v) for v in re.findall(r"\d+", m.group(1))]
    assert listed == ori_build.supported_lengths()


def test_version_and_defaults():
    assert "gfx950" in ori.ori_version()
    o = ori.ori_default_opts()
    assert o.tol == 1e-10 and o.max_iter == 1000 and o.precision == ori.ORI_FP64
    assert o.check_every == 1 and o.true_residual == 1 and o.graph == 1
    assert o.inner_tol == 1e-5 and o.max_outer == 10 and o.use_x0 == 0


@pytest.mark.parametrize("n", [1, 2, 3, 16, 64, 128, 256, 512])
def test_workspace_bytes_supported(n):
    b = ori.ori_workspace_bytes(n)
    assert b >= 6 * n ** 3 * 16 + 8 * n ** 3 * 16
    # FP64-only provisioning is smaller
    assert ori.ori_workspace_bytes(n, ori.ORI_PROVISION_FP64) < b


def test_workspace_bytes_metric_size_fits_hbm():
    # n = 256 (16.8 M unknowns): a few GB; n = 512 stays far below 288 GB
    assert ori.ori_workspace_bytes(256) < 8e9
    assert ori.ori_workspace_bytes(512) < 60e9
    # a batch of 32 right-hand sides at n = 64 shares the operator buffers
    one, many = ori.ori_workspace_bytes(64), ori.ori_workspace_bytes(64, nrhs=32)
    assert one < many < 32 * one


@pytest.mark.parametrize("n,status", [(0, ori.ORI_ERR_INVALID_ARG), (-3, ori.ORI_ERR_INVALID_ARG),
                                      (513, ori.ORI_ERR_UNSUPPORTED), (1024, ori.ORI_ERR_UNSUPPORTED)])
def test_bad_grid_rejected_on_host(n, status):
    with pytest.raises(ori.OriError) as e:
        ori.ori_workspace_bytes(n)
    assert e.value.status == status
    assert ori.ori_last_error() != "no error"


@pytest.mark.parametrize("n,L", [(1, 2), (7, 16), (8, 16), (9, 20), (11, 24), (14, 32), (33, 80), (100, 256),
                                 (256, 512), (257, 1024), (500, 1024), (512, 1024)])
def test_any_n_up_to_512_pads_to_a_planned_length(n, L):
    # every n <= 512 is accepted: the padded length is the shortest planned
    # L >= 2n - 1 (the work arrays hold n*n*L + n*L*L elements per right-hand
    # side and the spectrum octant (L/2 + 1)^3)
    b = ori.ori_workspace_bytes(n, ori.ORI_PROVISION_FP64)
    kp = L // 2 + 1
    assert b >= (n * n * L + n * L * L) * 16 + kp ** 3 * 16 + 8 * n ** 3 * 16
    assert b < (n * n * L + n * L * L) * 16 + kp ** 3 * 16 + 12 * n ** 3 * 16 + (1 << 24)


def test_bad_side_and_null_grid():
    lib = ori.lib()
    g = ori._grid(8, side=float("nan"))
    out = ctypes.c_int64()
    assert lib.ori_workspace_bytes(ctypes.byref(g), 1, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_workspace_bytes(None, 1, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    g = ori._grid(8, side=-1.0)
    assert lib.ori_workspace_bytes(ctypes.byref(g), 1, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    g = ori._grid(8, origin=(0.0, float("inf"), 0.0))
    assert lib.ori_workspace_bytes(ctypes.byref(g), 1, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    g = ori._grid(8)
    assert lib.ori_workspace_bytes(ctypes.byref(g), 0, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_workspace_bytes(ctypes.byref(g), 4096, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG


def test_memory_limit_rejected_before_any_device_call():
    # n = 512 under a 1 GB cap: ORI_ERR_OUT_OF_MEMORY, decided on the host
    lib = ori.lib()
    h = ctypes.c_void_p()
    g = ori._grid(512)
    st = lib.ori_create(ctypes.byref(g), 1, 3, 1 << 30, None, ctypes.byref(h))
    assert st == ori.ORI_ERR_OUT_OF_MEMORY
    assert h.value is None
    assert "exceeds the limit" in ori.ori_last_error()


def test_null_context_calls_fail_cleanly():
    lib = ori.lib()
    assert lib.ori_load(None, 1.0, None, None, None) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_solve(None, None, None, None) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_matvec(None, 0, 0, None, None) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_profile_enable(None, 1) == ori.ORI_ERR_INVALID_ARG
    lib.ori_destroy(None)
    assert lib.ori_create(None, 1, 3, 0, None, None) == ori.ORI_ERR_INVALID_ARG
    assert lib.ori_batch_info(None, 0, None) == ori.ORI_ERR_INVALID_ARG


def test_no_oracle_in_product_path():
    # the library and its binding never reach the CPU oracle
    pkg = os.path.join(ROOT, "paper_1602_04691_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


@pytest.mark.parametrize("nrhs", [0, -1, 1 << 20])
def test_bad_batch_size_rejected_on_host(nrhs):
    lib = ori.lib()
    g = ori._grid(8)
    out = ctypes.c_int64()
    assert lib.ori_workspace_bytes(ctypes.byref(g), nrhs, 3, ctypes.byref(out)) == ori.ORI_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.ori_create(ctypes.byref(g), nrhs, 3, 0, None, ctypes.byref(h)) == ori.ORI_ERR_INVALID_ARG
    assert h.value is None


_CTYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}


def _header_structs():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(ori_[a-z_]+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            m = re.fullmatch(r"(\w+)\s+(\w+)(?:\[(\d+)\])?", decl)
            assert m, (name, decl)
            ty = _CTYPES[m.group(1)]
            fields.append((m.group(2), ty * int(m.group(3)) if m.group(3) else ty))
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyname", [("ori_grid", "Grid"), ("ori_solve_opts", "SolveOpts"),
                                          ("ori_solve_info", "SolveInfo"), ("ori_layout", "Layout")])
def test_binding_structs_match_header(cname, pyname):
    # the ctypes mirrors have the header's fields, in order, at the same offsets
    fields = _header_structs()[cname]

    class FromHeader(ctypes.Structure):
        _fields_ = fields

    mirror = getattr(ori, pyname)
    assert [f for f, _ in mirror._fields_] == [f for f, _ in fields]
    assert ctypes.sizeof(mirror) == ctypes.sizeof(FromHeader)
    for f, _ in fields:
        assert getattr(mirror, f).offset == getattr(FromHeader, f).offset, f
        assert getattr(mirror, f).size == getattr(FromHeader, f).size, f
