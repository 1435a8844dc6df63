"""The C ABI library loads and exports every symbol include/dgdft_alb.h
declares; argument validation that needs no device runs on the CPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgdft_alb.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|void|const char\s*\*)\s*(dgdft_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("dgdft_alb_create", "dgdft_alb_solve", "dgdft_alb_apply_h", "dgdft_alb_destroy",
              "dgdft_alb_last_error", "dgdft_strerror", "dgdft_alb_sizes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1506_08147_amd as pkg
    lib = pkg.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(pkg.EXPORTS)


def test_strerror():
    import paper_1506_08147_amd as pkg
    lib = pkg.load_library()
    assert lib.dgdft_strerror(0) == b"success"
    assert b"rank" in lib.dgdft_strerror(-5)


def _create(grid, box, J, **kw):
    import paper_1506_08147_amd as pkg
    return pkg.ALB([grid], [box], [J], **kw)


def test_create_rejects_radix_seven_grid():
    import paper_1506_08147_amd as pkg
    with pytest.raises(pkg.DGDFTError) as ei:
        _create((14, 12, 12), (5.0, 5.0, 5.0), 4)
    assert ei.value.code == -2


def test_create_rejects_bad_shapes():
    import paper_1506_08147_amd as pkg
    for grid, box, J, kw in [((12, 12, 12), (5.0, -1.0, 5.0), 4, {}),
                             ((12, 12, 12), (5.0, 5.0, 5.0), 0, {}),
                             ((1, 12, 12), (5.0, 5.0, 5.0), 2, {}),
                             ((12, 12, 12), (5.0, 5.0, 5.0), 4,
                              dict(elem_lo=[(0, 0, 0)], elem_hi=[(13, 4, 4)])),
                             ((12, 12, 12), (5.0, 5.0, 5.0), 4, dict(n_alb=[5]))]:
        with pytest.raises(pkg.DGDFTError) as ei:
            _create(grid, box, J, **kw)
        assert ei.value.code == -1


def test_create_rejects_tiles_above_lds():
    import paper_1506_08147_amd as pkg
    with pytest.raises(pkg.DGDFTError) as ei:
        _create((96, 96, 8), (40.0, 40.0, 3.0), 4)
    assert ei.value.code == -2


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1506_08147_amd.binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(b.LibraryMissing):
        b.load_library()


def test_binding_structs_match_the_header(tmp_path):
    """Field offsets and sizes of the ctypes mirrors equal those of the C
    structs (the header compiled with the host C compiler)."""
    import shutil
    import subprocess
    import paper_1506_08147_amd.binding as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"dgdft_alb_opts": b.Opts, "dgdft_kb": b.KB, "dgdft_alb_stats": b.Stats,
             "dgdft_pairs": b.Pairs, "dgdft_train_opts": b.TrainOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n"):
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
