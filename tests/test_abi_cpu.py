"""The C ABI on the CPU: the library loads, exports every function the header
declares, and rejects bad arguments before touching the device."""
import os
import re
import subprocess

import numpy as np
import pytest

import graphgen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcmf.h")
LIB = os.path.join(ROOT, "paper_2308_01037_amd", "libmcmf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmcmf.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcmf_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = _declared()
    assert {"mcmf_graph_create", "mcmf_diag", "mcmf_action"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mcmf_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    from paper_2308_01037_amd import mcmf as M
    assert sorted(M.EXPORTED) == names


def test_status_strings():
    from paper_2308_01037_amd import mcmf as M
    assert M.mcmf_status_string(M.MCMF_OK) == "MCMF_OK"
    assert M.mcmf_status_string(M.MCMF_E_NOT_SYMMETRIC) == "MCMF_E_NOT_SYMMETRIC"
    assert M.mcmf_status_string(99) == "MCMF_E_UNKNOWN"


def test_argument_errors_need_no_device():
    import ctypes
    from paper_2308_01037_amd import mcmf as M
    g = G.path(5)
    lib = M._lib
    assert lib.mcmf_graph_create(5, g.row_ptr.ctypes.data, g.col.ctypes.data, None, 1, None) == M.MCMF_E_ARG
    out = ctypes.c_void_p()
    assert lib.mcmf_graph_create(-1, g.row_ptr.ctypes.data, g.col.ctypes.data, None, 1,
                                 ctypes.byref(out)) == M.MCMF_E_ARG
    assert lib.mcmf_graph_create(5, None, g.col.ctypes.data, None, 1, ctypes.byref(out)) == M.MCMF_E_ARG
    assert lib.mcmf_graph_create(5, g.row_ptr.ctypes.data, g.col.ctypes.data, None, 64,
                                 ctypes.byref(out)) == M.MCMF_E_ARG
    rp = g.row_ptr.copy()
    rp[0] = 1
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_graph_create(5, rp, g.col)
    assert e.value.status == M.MCMF_E_CSR and "row_ptr[0]" in M.mcmf_last_error()
    big = np.array([0, 2**32], dtype=np.int64)
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_graph_create(1, big, np.zeros(1, np.int32))
    assert e.value.status == M.MCMF_E_UNSUPPORTED
    y = np.zeros(5)
    f = M.make_fn()
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_action(None, f, np.ones(5), 10, 5, None, y)
    assert e.value.status == M.MCMF_E_ARG and "graph" in M.mcmf_last_error()
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_diag(None, f, None, 0, 10, 5, None, y)
    assert e.value.status == M.MCMF_E_ARG
    assert np.all(y == 0)


def test_import_fails_loudly_without_library(tmp_path):
    # A copy of the binding next to no library must refuse to import.
    import shutil
    import sys
    pkg = tmp_path / "pkgcopy"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2308_01037_amd", "mcmf.py"), pkg / "mcmf.py")
    code = f"import sys; sys.path.insert(0, {str(pkg)!r}); import mcmf"
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert res.returncode != 0 and "libmcmf.so is missing" in res.stderr


def test_struct_layouts_match_header(tmp_path):
    # The ctypes mirrors of the public structs must have the C layout.
    from paper_2308_01037_amd import mcmf as M
    structs = {"mcmf_fn": M.mcmf_fn, "mcmf_opts": M.mcmf_opts, "mcmf_stats": M.mcmf_stats,
               "mcmf_request": M.mcmf_request, "mcmf_batch_opts": M.mcmf_batch_opts,
               "mcmf_server_opts": M.mcmf_server_opts, "mcmf_ticket_info": M.mcmf_ticket_info,
               "mcmf_server_stats": M.mcmf_server_stats, "mcmf_tuning": M.mcmf_tuning}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mcmf.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    import ctypes
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_batch_argument_errors_need_no_device():
    from paper_2308_01037_amd import mcmf as M
    f = M.make_fn()
    y = np.zeros(5)
    # An empty batch is a no-op.
    M.mcmf_batch([])
    bad = M.make_request(M.MCMF_REQ_ACTION, None, f, 5, 10, y, v=np.ones(5))
    ok_shape = M.make_request(M.MCMF_REQ_DIAG, None, f, 5, 10, y)
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_batch([bad, ok_shape])
    assert e.value.status == M.MCMF_E_ARG and bad.status == M.MCMF_E_ARG
    assert "graph" in M.mcmf_last_error()
    o = M.mcmf_batch_opts()
    o.reserved[2] = 1
    with pytest.raises(M.MCMFError) as e:
        M.mcmf_batch([bad], o)
    assert e.value.status == M.MCMF_E_ARG and "reserved" in M.mcmf_last_error()
    kind = M.make_request(7, None, f, 5, 10, y)
    with pytest.raises(M.MCMFError):
        M.mcmf_batch([kind])
    assert np.all(y == 0)


def test_server_argument_errors_need_no_device():
    import ctypes
    from paper_2308_01037_amd import mcmf as M
    lib = M._lib
    out = ctypes.c_void_p()
    assert lib.mcmf_server_create(None, None) == M.MCMF_E_ARG
    o = M.mcmf_server_opts()
    o.reserved[0] = 1
    assert lib.mcmf_server_create(ctypes.byref(o), ctypes.byref(out)) == M.MCMF_E_ARG
    o = M.mcmf_server_opts()
    o.n_streams = 17
    assert lib.mcmf_server_create(ctypes.byref(o), ctypes.byref(out)) == M.MCMF_E_ARG
    assert "n_streams" in M.mcmf_last_error()
    o = M.mcmf_server_opts()
    o.n_streams, o.max_large_in_flight = 2, 3
    assert lib.mcmf_server_create(ctypes.byref(o), ctypes.byref(out)) == M.MCMF_E_ARG
    assert "max_large_in_flight" in M.mcmf_last_error()
    o = M.mcmf_server_opts()
    o.max_batch = -1
    assert lib.mcmf_server_create(ctypes.byref(o), ctypes.byref(out)) == M.MCMF_E_ARG
    t = ctypes.c_uint64()
    assert lib.mcmf_server_submit(None, None, ctypes.byref(t)) == M.MCMF_E_ARG
    assert lib.mcmf_server_wait(None, 1, None) == M.MCMF_E_ARG
    assert lib.mcmf_server_query(None, None) == M.MCMF_E_ARG
    lib.mcmf_server_destroy(None)


def test_digraph_flag_errors_need_no_device():
    import ctypes
    from paper_2308_01037_amd import mcmf as M
    lib = M._lib
    out = ctypes.c_void_p()
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    assert lib.mcmf_graph_create(2, rp.ctypes.data, col.ctypes.data, None,
                                 M.MCMF_DIGRAPH | M.MCMF_SYMMETRIC, ctypes.byref(out)) == M.MCMF_E_ARG
    assert lib.mcmf_graph_create(2, rp.ctypes.data, col.ctypes.data, None, 8,
                                 ctypes.byref(out)) == M.MCMF_E_ARG
    bad = np.array([1, 2], dtype=np.int32)
    assert lib.mcmf_graph_create(2, rp.ctypes.data, bad.ctypes.data, None, M.MCMF_DIGRAPH,
                                 ctypes.byref(out)) == M.MCMF_E_CSR
    assert "outside" in M.mcmf_last_error()
    down = np.array([0, 2, 1], dtype=np.int64)
    assert lib.mcmf_graph_create(2, down.ctypes.data, col.ctypes.data, None, M.MCMF_DIGRAPH,
                                 ctypes.byref(out)) == M.MCMF_E_CSR
