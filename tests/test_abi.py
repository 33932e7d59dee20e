"""CPU-side checks of the C ABI: the in-tree library loads and exports every
function that include/abft.h declares (no compute call needs a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "abft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\bint\s+(abft_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for must in ["abft_potrf", "abft_getrf", "abft_geqrf", "abft_encode", "abft_verify", "abft_gesv_mp",
                 "abft_posv_mp", "abft_potrf_batched", "abft_getrf_batched", "abft_workspace_size"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2301_03166_amd import abft
    lib = ctypes.CDLL(abft.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_struct_sizes_match_header_layout():
    from paper_2301_03166_amd import abft
    # abft_report: 5 int64 + 2 int32 + double + 2 int32 + 16 events of 24 bytes
    assert ctypes.sizeof(abft.Report) == 5 * 8 + 8 + 8 + 8 + 16 * 24
    assert ctypes.sizeof(abft.Fault) == 32
    assert ctypes.sizeof(abft.Opts) == 32
    assert ctypes.sizeof(abft.IRReport) == 48
