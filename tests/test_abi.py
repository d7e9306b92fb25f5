"""The C-ABI library loads on a machine without a GPU and exports every
function include/bamg.h declares; host-side defaults match the header."""
import os
import re

from paper_1004_1451_amd import bamg as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bamg_[a-z_]+)\s*\(", src)))


def test_header_functions_are_exported():
    lib = B.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTS) == names


def test_default_options():
    o = B.default_options()
    assert (o.levels, o.coarse_max, o.nu_setup, o.nu_pre, o.nu_post) == (0, 1024, 4, 2, 2)
    assert o.omega == 0.7 and o.caliber == 4 and o.n_eig == 6 and o.gmres_m == 50
    assert o.precision == B.FP64 and o.interp == B.INTERP_LS


def test_null_arguments_fail_without_gpu():
    import ctypes as C
    lib = B.load()
    h = C.c_void_p()
    rc = lib.bamg_setup(4, None, None, None, B.Grid(2, 2, 0), 1, None, None, C.byref(h))
    assert rc == B.EINVAL
    assert b"NULL" in lib.bamg_last_error()
    assert lib.bamg_free(None) == B.OK
    assert lib.bamg_solve(None, None, 1e-10, 1, 0, None) == B.EINVAL


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors have the size and field offsets the C compiler gives
    import ctypes as C
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    structs = {"bamg_grid": B.Grid, "bamg_options": B.Options, "bamg_solve_info": B.SolveInfo,
               "bamg_stats": B.Stats, "bamg_level_info": B.LevelInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bamg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in out:
        if not line:
            continue
        cname, what, val = line.split()
        py = structs[cname]
        got = C.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), (cname, what, got, val)


def test_size_limit_is_refused_before_any_launch():
    # n (r + 8) >= 2^31 (row, column) pairs: refused on the host with
    # EUNSUPPORTED before any device work (dummy non-NULL pointers are never
    # dereferenced)
    import ctypes as C
    lib = B.load()
    h = C.c_void_p()
    fake = C.c_void_p(16)
    n = (1 << 30) - 4
    ny = 2
    rc = lib.bamg_setup(n, fake, fake, fake, B.Grid(n // ny, ny, 0), 12, None, None, C.byref(h))
    assert rc == B.EUNSUPPORTED
    assert b"2^31" in lib.bamg_last_error()
