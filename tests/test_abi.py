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


def _header_layout(tmp_path):
    """sizeof / offsetof of the header's structs, from the C compiler itself."""
    import subprocess
    fields = {"abft_opts": ["nb", "protect", "tau_scale", "faults", "nfaults", "flags", "wgs_per_cu"],
              "abft_report": ["flagged_tiles", "first_flag_iter", "status", "max_ratio", "nev", "ev"],
              "abft_fault": ["iter", "target", "row", "col", "bit", "matrix"],
              "abft_event": [], "abft_ir_report": [], "abft_profile": []}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "abft.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


def test_binding_struct_layouts_match_header(tmp_path):
    from paper_2301_03166_amd import abft
    lay = _header_layout(tmp_path)
    pairs = {"abft_opts": abft.Opts, "abft_report": abft.Report, "abft_fault": abft.Fault,
             "abft_ir_report": abft.IRReport, "abft_profile": abft.Profile}
    for cname, py in pairs.items():
        assert ctypes.sizeof(py) == lay[cname], cname
        for key, off in lay.items():
            if key.startswith(cname + "."):
                assert getattr(py, key.split(".")[1]).offset == off, key


def test_autotune_table_lookup(tmp_path):
    """Lookups read the tuned table by (operation, size class) and fall back
    to the defaults; a lookup never returns a block size above n."""
    from paper_2301_03166_amd import autotune
    assert autotune.size_class(1) == 1 and autotune.size_class(8192) == 8192 and autotune.size_class(8193) == 16384
    t = {"nb": {"getrf:8192": {"best": 384}}, "batched": {"potrf:f32": {"best": 2}}}
    assert autotune.lookup_nb("getrf", 8000, t) == 384
    assert autotune.lookup_nb("potrf", 8000, t) == autotune.default_nb("potrf", 8000)
    assert autotune.lookup_nb("geqrf", 100, t) == 100
    assert autotune.lookup_wgs("potrf", "f32", t) == 2 and autotune.lookup_wgs("getrf", "f64", t) == 1
    p = tmp_path / "t.json"
    autotune.save(t, str(p))
    assert autotune.load(str(p)) == t


def test_handle_calls_reject_null_handle():
    """Argument checks that need no device: a NULL handle is argument 1."""
    from paper_2301_03166_amd import abft
    L = abft.lib()
    assert L.abft_set_workspace(None, None, 0) == -1
    assert L.abft_report_fetch(None, None, None) == -1
    assert L.abft_set_stream(None, None) == -1
