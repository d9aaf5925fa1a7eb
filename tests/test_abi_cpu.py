"""The C-ABI library loads on the CPU and exports every declared entry point
(no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2310_13143_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(acopf_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(_abi.EXPORTS)


@pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.acopf_workspace_bytes.restype = ctypes.c_size_t
    lib.acopf_workspace_bytes.argtypes = [ctypes.c_int32] * 4
    assert lib.acopf_workspace_bytes(14, 20, 5, 1) > 0
    assert lib.acopf_workspace_bytes(0, 20, 5, 1) == 0
    assert lib.acopf_workspace_bytes(28, 40, 10, 2) > lib.acopf_workspace_bytes(14, 20, 5, 1)


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and member offsets of the ctypes mirrors equal the C compiler's."""
    import subprocess
    checks = {"acopf_grid": _abi.Grid, "acopf_iterate": _abi.Iterate, "acopf_admm_params": _abi.AdmmParams,
              "acopf_admm_result": _abi.AdmmResult, "acopf_admm_state": _abi.AdmmState,
              "acopf_sqp_params": _abi.SqpParams, "acopf_sqp_state": _abi.SqpState,
              "acopf_residuals_report": _abi.ResidualsReport}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "acopf_admm.h"', "int main(void) {"]
    for cname, py in checks.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for cname, py in checks.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)
