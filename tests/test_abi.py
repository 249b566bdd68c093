"""The C-ABI library loads, exports every symbol include/aqt.h declares, and the
binding's ctypes layouts match the C compiler's (no GPU work)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aqt.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1710_03431_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1710_03431_amd import build
        build.build()
    return binding.load_library()


def declared_symbols():
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"AQT_API\s+[\w\s\*]+?\b(aqt_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    from paper_1710_03431_amd import binding
    assert set(binding.EXPORTED) == set(names)


def test_version_call_needs_no_gpu(lib):
    assert lib.aqt_version() >= 10000


def test_struct_layouts_match_c(tmp_path):
    from paper_1710_03431_amd import binding
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "aqt.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(aqt_jump), sizeof(aqt_run_params),'
                   ' sizeof(aqt_outputs), offsetof(aqt_outputs, hist_lo), offsetof(aqt_outputs, final_state),'
                   ' offsetof(aqt_run_params, tile));return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(binding.Jump), ctypes.sizeof(binding.RunParams), ctypes.sizeof(binding.Outputs),
            binding.Outputs.hist_lo.offset, binding.Outputs.final_state.offset, binding.RunParams.tile.offset]
    assert got == want


def test_null_context_is_rejected(lib):
    assert lib.aqt_set_bath(None, 1e-4, 1.0, 1.0) == -1
    assert lib.aqt_run(None, None, None) == -1
    n = ctypes.c_int32(0)
    assert lib.aqt_bound_grid_points(None, 1.0, 11, ctypes.byref(n)) == -1 and n.value == 0
