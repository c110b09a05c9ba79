"""The C-ABI library builds, loads and exports every entry point that include/ccmc.h
declares (no GPU needed: no compute call is made here)."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "ccmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ccmc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for required in ("ccmc_init", "ccmc_step", "ccmc_energy", "ccmc_free", "ccmc_import", "ccmc_export",
                     "ccmc_export_spawns", "ccmc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1807_03749_amd import ccmc
    if not os.path.exists(ccmc.LIB_PATH):
        pytest.skip("libccmc.so not built (run __graft_entry__.build())")
    lib = C.CDLL(ccmc.LIB_PATH)
    for name in declared_entry_points():
        assert hasattr(lib, name), name
    assert sorted(ccmc.EXPORTED) == declared_entry_points()


def test_options_default_host_only():
    from paper_1807_03749_amd import ccmc
    if not os.path.exists(ccmc.LIB_PATH):
        pytest.skip("libccmc.so not built")
    o = ccmc.options()
    assert o.precision == ccmc.CCMC_FP64 and o.min_spawn_attempts == 1 and o.seed == 1234
    assert o.spawn_cutoff == 0.01 and o.occupation_threshold == 1.0 and o.noncomposite_threshold == 1.0


def test_library_has_no_oracle_dependency():
    """The product library and binding never reference the oracle."""
    for path in ("paper_1807_03749_amd/ccmc.py", "paper_1807_03749_amd/csrc/ccmc.hip",
                 "paper_1807_03749_amd/csrc/kernels.h", "paper_1807_03749_amd/csrc/device.h",
                 "paper_1807_03749_amd/csrc/primitives.h"):
        txt = open(os.path.join(ROOT, path)).read()
        assert "oracle" not in txt.lower().replace("oracle_", ""), path


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets that a C compiler
    gives the header's structures (a field added on one side only would shift the others)."""
    import shutil
    import subprocess

    from paper_1807_03749_amd import ccmc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"ccmc_system": ccmc.ccmc_system, "ccmc_integrals": ccmc.ccmc_integrals,
               "ccmc_options": ccmc.ccmc_options, "ccmc_stats": ccmc.ccmc_stats,
               "ccmc_shift_control": ccmc.ccmc_shift_control, "ccmc_kernel_time": ccmc.ccmc_kernel_time}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ccmc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
