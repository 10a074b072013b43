"""The C-ABI boundary without a GPU: libfgraft.so loads, exports every
function include/*.h declares, the Python binding covers exactly those
names, and the library references nothing of the oracle."""
import ctypes
import glob
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_30493_amd", "libfgraft.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*(fg_[A-Za-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("fg_workspace_size", "fg_roots", "fg_build_scaffold", "fg_harvest_block", "fg_merge_block",
                 "fg_finalize", "fg_build_graph", "fg_search", "fg_graph_hash", "fg_leaf_knn",
                 "fg_screen_copy", "fg_last_error"):
        assert must in names


def test_library_loads_and_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python __graft_entry__.py or build.py)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared_functions()) if getattr(lib, n, None) is None]
    assert not missing, missing


def test_binding_names_match_the_header():
    from paper_2609_30493_amd import fgraft as F
    assert set(F._SIGS) == declared_functions()


def test_library_does_not_reference_the_oracle():
    out = subprocess.run(["nm", "-D", LIB], capture_output=True, text=True, check=True).stdout
    assert "fgo_" not in out


def test_roots_without_gpu():
    """fg_roots is host-only: it runs without a device."""
    lib = ctypes.CDLL(LIB)
    roots = (ctypes.c_uint32 * 4)()
    rc = lib.fg_roots(ctypes.c_uint64(0), ctypes.c_int64(1000), ctypes.c_uint32(4), roots)
    assert rc == 0
    assert len(set(roots)) == 4 and all(r < 1000 for r in roots)
    assert lib.fg_roots(ctypes.c_uint64(0), ctypes.c_int64(3), ctypes.c_uint32(4), roots) == -1


def test_screen_row_bytes_without_gpu():
    """fg_screen_row_bytes is host-only: narrow rows are whole 128-byte
    lines holding the codes (bfloat16: 2d rounded up to 32; fp8: d rounded
    up to 16) and the 16-byte trailer, with less than a line to spare; bad
    kinds and sizes give 0."""
    lib = ctypes.CDLL(LIB)
    lib.fg_screen_row_bytes.restype = ctypes.c_int64
    lib.fg_screen_row_bytes.argtypes = [ctypes.c_int32, ctypes.c_uint32]
    for d in (68, 96, 100, 128, 256, 260, 512, 960, 1024):
        for kind, codes in ((1, (2 * d + 31) // 32 * 32), (2, (d + 15) // 16 * 16), (4, (d + 15) // 16 * 16)):
            rb = lib.fg_screen_row_bytes(d, kind)
            assert rb % 128 == 0 and codes + 16 <= rb < codes + 16 + 128, (d, kind, rb)
    assert lib.fg_screen_row_bytes(100, 1) == 256 and lib.fg_screen_row_bytes(100, 2) == 128
    assert lib.fg_screen_row_bytes(0, 1) == 0 and lib.fg_screen_row_bytes(100, 7) == 0
    assert lib.fg_screen_row_bytes(100, 3) == 0  # the split tiles have no narrow search copy
