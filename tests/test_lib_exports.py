"""The C-ABI library builds for gfx950, loads without a GPU, and exports every
function that include/chebdav.h declares (no compute calls here)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chebdav.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chebdav_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["chebdav_build_laplacian", "chebdav_filter", "chebdav_orthonormalize",
                     "chebdav_solve"]:
        assert required in names


def test_library_exports_every_declared_symbol(cd):
    lib = ctypes.CDLL(cd.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(cd.EXPORTED) == _declared()


def test_struct_layouts_match_header(cd, tmp_path):
    """The ctypes mirrors of chebdav_params / chebdav_stats / chebdav_iter_record have the C layout
    (checked by compiling the header with gcc)."""
    import subprocess
    fields_p = [f for f, _ in cd.Params._fields_]
    fields_s = [f for f, _ in cd.Stats._fields_]
    fields_r = [f for f, _ in cd.IterRecord._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "chebdav.h"', "int main(void){",
            'printf("%zu %zu %zu\\n", sizeof(chebdav_params), sizeof(chebdav_stats), sizeof(chebdav_iter_record));']
    prog += ['printf("%%zu\\n", offsetof(chebdav_params, %s));' % f for f in fields_p]
    prog += ['printf("%%zu\\n", offsetof(chebdav_stats, %s));' % f for f in fields_s]
    prog += ['printf("%%zu\\n", offsetof(chebdav_iter_record, %s));' % f for f in fields_r]
    prog += ["return 0;}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(cd.Params) and int(out[1]) == ctypes.sizeof(cd.Stats)
    assert int(out[2]) == ctypes.sizeof(cd.IterRecord)
    offs = [int(x) for x in out[3:]]
    want = [getattr(cd.Params, f).offset for f in fields_p] + [getattr(cd.Stats, f).offset for f in fields_s]
    want += [getattr(cd.IterRecord, f).offset for f in fields_r]
    assert offs == want


def test_last_error_callable_without_gpu(cd):
    assert isinstance(cd.last_error(), str)
