"""The C-ABI library loads and exports every function include/nmr.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmr.h")
LIB = os.path.join(ROOT, "paper_2102_11026_amd", "libnmr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s+([a-z_]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("decoder_jacobian_hessian", "cubature_force_stiffness", "reduced_newton_step", "step_many",
              "nmr_create", "nmr_instance_create"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    from paper_2102_11026_amd import nmr
    monkeypatch.setattr(nmr, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nmr, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        nmr.lib()


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
@pytest.mark.parametrize("c_name,py_name", [("nmr_mlp_desc", "MlpDesc"), ("nmr_problem", "ProblemDesc"),
                                            ("nmr_tile_choice", "TileChoice")])
def test_binding_structs_match_the_header(tmp_path, c_name, py_name):
    """Every struct the binding passes across the ABI has the header's size
    and, field by field, its offsets (compiled against include/nmr.h)."""
    from paper_2102_11026_amd import nmr
    py = getattr(nmr, py_name)
    fields = [f[0] for f in py._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"nmr.h\"\nint main(void) {\n"
                   f'  printf("%zu\\n", sizeof({c_name}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({c_name}, {f}));\n' for f in fields) + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(py), (c_name, out[0], ctypes.sizeof(py))
    assert out[1:] == [getattr(py, f).offset for f in fields], c_name
