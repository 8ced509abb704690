"""CPU-side checks of the C ABI: the library loads, exports every function
include/slaq.h declares, and rejects bad arguments on the host before any
device work (no GPU is touched by these calls)."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_2003_01282_amd import slaq as S

HEADER = Path(__file__).resolve().parents[1] / "include" / "slaq.h"


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(slaq_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_named_entry_points():
    names = declared_functions()
    for required in ("slaq_build_graph", "slaq_lanczos", "slaq_signature", "slaq_vnge", "slaq_ritz"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    for name in S.SIGNATURES:
        assert name in declared_functions(), name


def test_host_side_argument_errors():
    L = S.lib()
    b = ctypes.c_size_t()
    assert L.slaq_graph_scratch_bytes(0, 0, ctypes.byref(b)) == 1
    assert L.slaq_graph_scratch_bytes(10, -1, ctypes.byref(b)) == 1
    assert L.slaq_graph_scratch_bytes(10, 20, ctypes.byref(b)) == 0 and b.value > 0
    assert L.slaq_lanczos_workspace(None, 4, 4, ctypes.byref(b)) == 1
    h = ctypes.c_void_p()
    # NULL row_ptr: rejected before anything is enqueued
    assert L.slaq_build_graph(10, 20, None, None, None, 0, 0, None, None, 0, None, ctypes.byref(h)) == 1
    assert b"non-NULL" in L.slaq_last_error()
    assert L.slaq_ritz(None, None, None, 4, 4, None, None, None) == 1
    assert L.slaq_lanczos_noalloc(None, 4, 4, 1, None, None, None, None) == 1
    assert L.slaq_graph_set_cache_rows(None, 0) == 1
    assert L.slaq_graph_set_fused(None, -1) == 1
    assert L.slaq_graph_autotune(None, 4, 4, 1, None, None, None, None, 0, 1, None, None, None) == 1
    assert L.slaq_graph_settings(None, None, None, None, None) == 1
    assert L.slaq_signature(None, None, 4, 4, 10, None, 8, 0, None, None) == 1
    # bucket growth outside [1.25, 8], and a missing output, are refused first
    assert L.slaq_batch_plan_grown(1, None, None, None, None, None, 4, 4, 1, 1.0, None, 0, ctypes.byref(h)) == 1
    assert b"growth" in L.slaq_last_error()
    assert L.slaq_batch_autotune_edges(1, None, None, None, None, None, 4, 4, 1, None, 3, None, None, None,
                                       None) == 1


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        S.build_graph(torch.zeros(3, dtype=torch.int64), torch.zeros(2, dtype=torch.int32))


def test_missing_library_fails_loudly():
    # no fallback path: without libslaq.so every entry point raises
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from pathlib import Path\n"
            "from paper_2003_01282_amd import slaq as S\n"
            "S.LIB_PATH = Path('/nonexistent/libslaq.so')\n"
            "try:\n"
            "    S.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(3)\n") % str(HEADER.parents[1])
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "is missing" in r.stdout, (r.stdout, r.stderr)
