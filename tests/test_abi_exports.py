"""The C-ABI library loads and exports every entry point that
include/smpc.h declares (no compute call: runs without a GPU)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smpc.h")
LIB = os.path.join(ROOT, "paper_1604_01074_amd", "libsmpc.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\bint\s+(smpc_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("smpc_ctx_create", "smpc_sys_create", "smpc_tree_create", "smpc_tree_set_data",
                 "smpc_factor", "smpc_solve", "smpc_solve_batch", "smpc_solve_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1604_01074_amd.build import build

        build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1604_01074_amd import smpc

    assert sorted(smpc.EXPORTED) == _declared()
    for n in smpc.EXPORTED:
        assert callable(getattr(smpc, n, None)) or n == "smpc_last_error"


def test_chunk_length_query_runs_without_a_gpu():
    from paper_1604_01074_amd import smpc

    for precision in (32, 64):
        for which in (0, 1):
            lens = smpc.smpc_chunk_lengths(precision, which)
            assert len(lens) >= 1 and len(set(lens)) == len(lens)
            assert all(n in (4, 8, 16, 32) for n in lens)
    # the defaults come first
    assert smpc.smpc_chunk_lengths(32, 0)[0] == 16 and smpc.smpc_chunk_lengths(64, 1)[0] == 4
    for bad in ((16, 0), (32, 2)):
        try:
            smpc.smpc_chunk_lengths(*bad)
        except smpc.SmpcError as e:
            assert e.code == smpc.EINVAL
        else:
            raise AssertionError(bad)
