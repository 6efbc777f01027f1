"""The C-ABI library loads and exports every symbol include/cse.h declares
(no GPU needed), and the binding refuses to run without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cse.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cse_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    assert "cse_launch" in names and "cse_get_program" in names and "cse_ctx_create" in names
    from paper_2512_13365_amd import cse
    assert sorted(cse.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    from paper_2512_13365_amd import cse
    if not os.path.exists(cse.LIB_PATH):
        pytest.skip("libcse.so not built")
    lib = ctypes.CDLL(cse.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.cse_version() == 1


def test_cfg_struct_layout_matches_header(tmp_path):
    """The binding's cse_run_cfg has the C compiler's size and offsets."""
    import subprocess

    from paper_2512_13365_amd import cse
    fields = [f[0] for f in cse.CseRunCfg._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cse.h"\nint main(void){\n'
                   '  printf("%zu\\n", sizeof(cse_run_cfg));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(cse_run_cfg, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cse.CseRunCfg) == 104
    for f, off in zip(fields, vals[1:]):
        assert getattr(cse.CseRunCfg, f).offset == off, f


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2512_13365_amd import cse
    saved = cse._lib
    cse._lib = None
    try:
        with pytest.raises(RuntimeError):
            cse.load_library(str(tmp_path / "missing.so"))
    finally:
        cse._lib = saved


def test_driver_cfg_struct_layout_matches_header(tmp_path):
    """The binding's cse_driver_cfg has the C compiler's size and offsets."""
    import subprocess

    from paper_2512_13365_amd import cse
    fields = [f[0] for f in cse.CseDriverCfg._fields_]
    src = tmp_path / "dlayout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "cse.h"\nint main(void){\n'
                   '  printf("%zu\\n", sizeof(cse_driver_cfg));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(cse_driver_cfg, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "dlayout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cse.CseDriverCfg) == 16
    for f, off in zip(fields, vals[1:]):
        assert getattr(cse.CseDriverCfg, f).offset == off, f


def test_binding_constants_match_header():
    """CSE_LAYOUT_*, CSE_COUNT_* and CSE_JOB_* of the binding equal the header's."""
    from paper_2512_13365_amd import cse
    defs = dict(re.findall(r"#define\s+(CSE_[A-Z_]+)\s+(-?\d+)", open(HEADER).read()))
    names = [n for n in defs if n.startswith(("CSE_LAYOUT_", "CSE_COUNT_", "CSE_JOB_"))]
    assert len(names) >= 9
    for n in names:
        assert getattr(cse, n) == int(defs[n]), n
    codes = dict(re.findall(r"#define\s+(CSE_OK|CSE_E[A-Z]+)\s+\(?(-?\d+)\)?", open(HEADER).read()))
    assert len(codes) == 8
    assert {int(v): k for k, v in codes.items()} == cse.STATUS


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_null_handles_rejected_before_any_device_call():
    """Every entry point that takes a context or a server returns CSE_EINVAL
    for a null one, before any HIP call (so this runs without a GPU), and the
    error text of a null context is defined."""
    from paper_2512_13365_amd import cse
    if not os.path.exists(cse.LIB_PATH):
        pytest.skip("libcse.so not built")
    L = cse.load_library()
    skip = {"cse_version", "cse_ctx_create", "cse_ctx_destroy", "cse_last_error", "cse_server_destroy"}
    pointer_like = (ctypes.c_void_p, ctypes.c_char_p)
    checked = 0
    for name in cse.EXPORTS:
        if name in skip:
            continue
        fn = getattr(L, name)
        assert fn.argtypes, f"{name} has no declared argument types"
        args = [0 if isinstance(t, type) and issubclass(t, ctypes._SimpleCData) and t not in pointer_like
                else None for t in fn.argtypes]
        assert fn(*args) == -1, name
        checked += 1
    assert checked == len(cse.EXPORTS) - len(skip)
    assert L.cse_last_error(None) == b"null context"
    L.cse_server_destroy(None)


def test_workload_inputs_match_persisted_digests():
    """Every workload's inputs regenerate to the sha256 persisted beside the
    generator (a changed numpy stream or generator would change the inputs
    of every parity test and measurement silently)."""
    from paper_2512_13365_amd import workloads
    stored = workloads.stored_digests()
    assert len(stored) == len(workloads.WORKLOADS)
    for fn in workloads.WORKLOADS.values():
        wl = fn()
        assert stored[wl.name] == workloads.workload_digest(wl), wl.name
