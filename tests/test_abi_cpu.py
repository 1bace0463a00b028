"""Host-side checks of the C-ABI library (no GPU needed): it loads, and it exports every
function include/klecgc.h declares; the ctypes structs match the header's layouts."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "klecgc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_method_entry_points():
    names = declared_functions()
    for required in ("kle_build", "gpc_fit", "gpc_predict", "fine_propagate", "cgc_diag_solve",
                     "parareal_solve", "kle_synthesize", "klecgc_create", "klecgc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2510_26180_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libklecgc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.SIGNATURES) == set(declared_functions())
    assert lib.klecgc_version and ctypes.cast(lib.klecgc_version, ctypes.c_void_p).value


def test_struct_layouts_match_the_c_compiler(tmp_path):
    from paper_2510_26180_amd import _lib
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    fields_p = [f for f, _ in _lib.Problem._fields_]
    fields_k = [f for f, _ in _lib.KleDesc._fields_]
    fields_t = [f for f, _ in _lib.Task._fields_]
    fields_u = [f for f, _ in _lib.Tuning._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "klecgc.h"', "int main(void){"]
    src.append('printf("%zu\\n", sizeof(klecgc_problem));')
    src += ['printf("%%zu\\n", offsetof(klecgc_problem, %s));' % f for f in fields_p]
    src.append('printf("%zu\\n", sizeof(klecgc_kle_desc));')
    src += ['printf("%%zu\\n", offsetof(klecgc_kle_desc, %s));' % f for f in fields_k]
    src.append('printf("%zu\\n", sizeof(klecgc_task));')
    src += ['printf("%%zu\\n", offsetof(klecgc_task, %s));' % f for f in fields_t]
    src.append('printf("%zu\\n", sizeof(klecgc_tuning));')
    src += ['printf("%%zu\\n", offsetof(klecgc_tuning, %s));' % f for f in fields_u]
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(_lib.Problem)] + [getattr(_lib.Problem, f).offset for f in fields_p]
    want += [ctypes.sizeof(_lib.KleDesc)] + [getattr(_lib.KleDesc, f).offset for f in fields_k]
    want += [ctypes.sizeof(_lib.Task)] + [getattr(_lib.Task, f).offset for f in fields_t]
    want += [ctypes.sizeof(_lib.Tuning)] + [getattr(_lib.Tuning, f).offset for f in fields_u]
    assert vals == want


def test_missing_library_fails_loudly(tmp_path):
    from paper_2510_26180_amd import _lib
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved
