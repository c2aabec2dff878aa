"""CPU checks of the C-ABI library: it loads without a GPU and exports every
entry point that include/sgw.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgw.h")
LIB = os.path.join(ROOT, "paper_2601_21005_amd", "libsgw.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgw_[a-zA-Z_0-9]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    from paper_2601_21005_amd import sgw
    assert declared() == sorted(sgw.EXPORTS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_2601_21005_amd import sgw
    monkeypatch.setattr(sgw, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(sgw, "_lib", None)
    with pytest.raises(ImportError):
        sgw.load()


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the field offsets the C compiler gives the
    structs of include/sgw.h."""
    import shutil
    import subprocess
    from paper_2601_21005_amd import sgw
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    structs = {"sgw_grid": sgw.SgwGrid, "sgw_projectors": sgw.SgwProjectors,
               "sgw_tdh_state": sgw.SgwTdhState, "sgw_sigma_params": sgw.SgwSigmaParams,
               "sgw_batch_item": sgw.SgwBatchItem, "sgw_cv_result": sgw.SgwCvResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.split("\n"):
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_max_states_matches_header():
    import re
    from paper_2601_21005_amd import sgw
    m = re.search(r"#define\s+SGW_MAX_STATES\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == sgw.SGW_MAX_STATES


def test_timer_bits_match_header():
    import re
    from paper_2601_21005_amd import sgw
    text = open(HEADER).read()
    for name in ("SGW_TIMER_CHEB_PLANE", "SGW_TIMER_KB_SCATTER"):
        m = re.search(r"#define\s+%s\s+(\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(sgw, name), name
