"""The C-ABI library builds, loads and exports every declared entry point (CPU only)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfairsc.h")
LIB = os.path.join(ROOT, "paper_2210_16435_amd", "libsfairsc.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfairsc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__

        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("sfairsc_graph_create", "sfairsc_eigs", "sfairsc_labels", "sfairsc_eigsum_backward",
                 "sfairsc_graph_destroy", "sfairsc_last_error", "sfairsc_apply_operator"):
        assert need in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_2210_16435_amd._lib import PROTOTYPES

    assert sorted(PROTOTYPES) == _declared()


def test_struct_layouts_match_header(tmp_path):
    # the Python mirrors of the option/info structs agree with the C compiler
    import shutil
    import subprocess

    from paper_2210_16435_amd import _lib as L

    if shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no C compiler / ROCm headers")
    src = tmp_path / "sz.c"
    fields = {
        "sfairsc_eigs_opts": (L.EigsOpts, ["seed", "sigma", "x0", "b0"]),
        "sfairsc_graph_stats": (L.GraphStats, ["sigma", "max_degree"]),
        "sfairsc_eigs_info": (L.EigsInfo, ["operator_applies", "spmm_ms", "max_rel_residual", "phase1_ms", "rr_ms",
                                            "operator_ms", "restart_ms", "degenerate", "restarts_unpredicted"]),
        "sfairsc_batch_info": (L.BatchInfo, ["batch_status", "double_spmm", "converged", "max_rel_residual",
                                             "graph_ms", "batch_ms", "phase_ms"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sfairsc.h"', "int main(void){"]
    for st, (_, fl) in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("%zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for st, (cls, fl) in fields.items():
        want.append(ctypes.sizeof(cls))
        for f in fl:
            want.append(getattr(cls, f).offset)
    assert got == want


def test_host_only_calls(lib):
    lib.sfairsc_version.restype = ctypes.c_char_p
    assert b"sfairsc" in lib.sfairsc_version()
    lib.sfairsc_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.sfairsc_last_error(), bytes)
    # argument validation happens before any device work
    lib.sfairsc_graph_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    rc = lib.sfairsc_graph_create(ctypes.byref(out), ctypes.c_int64(0), ctypes.c_int64(0), None, None, None, 1,
                                  None, 2, 0, None)
    assert rc == -1 and not out.value
    lib.sfairsc_graph_query.restype = ctypes.c_int
    assert lib.sfairsc_graph_query(None, None) == -1
    assert lib.sfairsc_eigs(None, 1, ctypes.c_double(1e-8), 0, None, None, None, None, None) == -1


def test_tuning_table_roundtrip(tmp_path):
    # the tuning table's file format, lookups and defaults are host-only
    import json

    import paper_2210_16435_amd as sf

    src = tmp_path / "table.json"
    src.write_text(json.dumps({
        "format": "sfairsc-tuning-1",
        "entries": [
            {"n_log2": 13, "degree_bucket": 2, "k_bucket": 1, "double_spmm": 0, "normalized": 0,
             "block_width": 16, "max_basis": 64, "spmm_rows": 2, "ms": 3.5},
            {"n_log2": 10, "degree_bucket": 0, "k_bucket": 0, "double_spmm": 1, "normalized": 1,
             "block_width": 4, "max_basis": 24, "spmm_rows": 8, "ms": 0.5},
        ],
    }))
    try:
        sf.tuning_load(str(src))
        assert sf.tuning_size() == 2
        # n = 10000 -> floor(log2) = 13; degree 40 -> bucket 2; k = 6 -> bucket 1; mixed
        assert sf.tuning_lookup(10000, 400000, 6, "mixed", False, 1e-6) == (16, 64, 2, True)
        # the same shape in double precision is not in the table: built-in rule
        b, m, r, hit = sf.tuning_lookup(10000, 400000, 6, "fp64", False, 1e-6)
        assert not hit and b == 8 and m % b == 0 and 6 + 1 + b <= m <= 80
        # a tolerance below the float floor selects double products
        assert sf.tuning_lookup(1500, 15000, 3, "mixed", True, 1e-9) == (4, 24, 8, True)
        out = tmp_path / "saved.json"
        sf.tuning_save(str(out))
        saved = json.loads(out.read_text())["entries"]
        assert len(saved) == 2
        key = {(e["n_log2"], e["double_spmm"]): e for e in saved}
        assert key[(13, 0)]["block_width"] == 16 and key[(13, 0)]["spmm_rows"] == 2
        assert key[(10, 1)]["max_basis"] == 24 and key[(10, 1)]["normalized"] == 1
        bad = tmp_path / "bad.json"
        bad.write_text('{"entries": [{"n_log2": 3}]}')
        with pytest.raises(sf.SfairscError):
            sf.tuning_load(str(bad))
    finally:
        sf.tuning_clear()
    assert sf.tuning_size() == 0
    assert sf.tuning_lookup(10000, 400000, 6, "mixed", False, 1e-6)[3] is False
