"""C ABI checks that need no GPU: the library loads, exports every function kcore.h declares,
and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "kcore.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(kcore_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("kcore_decompose", "kcore_decompose_ex", "kcore_decompose_batched",
                 "kcore_submit", "kcore_poll", "kcore_server_create", "kcore_server_destroy",
                 "kcore_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2502_08042_amd as K
    lib = ctypes.CDLL(K.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in kcore.h but not exported"
        assert name in K.SIGNATURES, f"{name} has no binding signature"


def test_struct_layouts_match_header(tmp_path):
    """Every field of the binding's ctypes structures sits at the offset the C compiler gives the
    header's field of the same name, and the sizes agree (gcc compiles a probe of kcore.h)."""
    import shutil
    import subprocess
    import paper_2502_08042_amd as K
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"kcore_options": K.Options, "kcore_stats": K.Stats,
               "kcore_server_config": K.ServerConfig, "kcore_request_stats": K.RequestStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kcore.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    r = subprocess.run(["gcc", "-x", "c", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0 and "hip_runtime_api.h" in r.stderr:
        pytest.skip("HIP headers not available")
    assert r.returncode == 0, r.stderr
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_argument_errors_without_device_work():
    import paper_2502_08042_amd as K
    lib = K.lib()
    one = np.zeros(2, dtype=np.int64)
    # negative n, n beyond the int32 id range: rejected before any HIP call
    assert lib.kcore_decompose(one.ctypes.data, None, -1, None, None) == -1
    assert "negative" in K.last_error()
    assert lib.kcore_decompose(one.ctypes.data, None, 1 << 31, None, None) == -1
    # n == 0 is a no-op
    assert lib.kcore_decompose(None, None, 0, None, None) == 0
    # bad options
    o = K.Options()
    o.mode = 7
    assert lib.kcore_decompose_ex(one.ctypes.data, None, 0, None, None, ctypes.byref(o), None) == -1
    o = K.Options()
    o.tile_edges = 100
    assert lib.kcore_decompose_ex(one.ctypes.data, None, 0, None, None, ctypes.byref(o), None) == -1
    o = K.Options()
    o.block_queue = 2000
    assert lib.kcore_decompose_ex(one.ctypes.data, None, 0, None, None, ctypes.byref(o), None) == -1
    o = K.Options()
    o.tail = -2
    assert lib.kcore_decompose_ex(one.ctypes.data, None, 0, None, None, ctypes.byref(o), None) == -1
    # k-core query: same argument checks
    assert lib.kcore_kcore_subgraph(one.ctypes.data, None, -1, 3, None, None, None, None) == -1
    assert lib.kcore_kcore_subgraph(None, None, 0, 3, None, None, None, None) == 0
    # batched: negative sizes, empty batch
    assert lib.kcore_decompose_batched(None, None, None, -1, 0, None, None) == -1
    assert lib.kcore_decompose_batched(None, None, None, 0, 0, None, None) == 0
    # server calls on a null handle
    t = ctypes.c_uint64(0)
    assert lib.kcore_submit(None, one.ctypes.data, None, 1, ctypes.byref(t)) == -1
    assert lib.kcore_poll(None, 1, None, None) == -1
    assert lib.kcore_cancel(None, 1) == -1
    lib.kcore_server_destroy(None)
    # server configuration: negative fields are refused before any device is touched
    for field in ("max_inflight", "max_large_inflight", "large_vertices", "max_batch_vertices"):
        cfg = K.ServerConfig()
        setattr(cfg, field, -1)
        assert not lib.kcore_server_create(ctypes.byref(cfg))
        assert "negative" in K.last_error()
    assert lib.kcore_version() >= 10000


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import importlib.util
    import shutil
    pkg = tmp_path / "pkgcopy"
    shutil.copytree(os.path.join(ROOT, "paper_2502_08042_amd"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    spec = importlib.util.spec_from_file_location("kcore_nolib", pkg / "__init__.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError, match="no fallback"):
        spec.loader.exec_module(mod)


def test_one_hip_runtime_in_process():
    """Importing the binding before PyTorch must still leave a single HIP runtime mapped: PyTorch's
    copy and the system's share a soname, and two runtimes in one process see no device."""
    import subprocess
    import sys
    code = ("import paper_2502_08042_amd, torch\n"
            "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(paths))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
