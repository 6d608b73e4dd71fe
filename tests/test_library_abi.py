"""The C-ABI library loads and exports every entry point declared in include/*.h
(CPU only: nothing is called that needs a GPU)."""
import ctypes
import glob
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2204_14167_amd import discos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(discos_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("discos_create", "discos_destroy", "discos_spread", "discos_solve_poisson",
                     "discos_set_hydro_kernel", "discos_spread_force_species",
                     "discos_interpolate_vel_species",
                     "discos_interpolate", "discos_near_field", "discos_step", "discos_check",
                     "discos_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(discos.LIB_PATH):
        pytest.fail("libdiscos.so not built (python -m paper_2204_14167_amd.build)")
    lib = ctypes.CDLL(discos.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _c_layout(struct, members):
    """offsetof of each member and sizeof, as gcc lays out the header's struct."""
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"discos.h\"\nint main(void) {\n"
    for m in members:
        src += f'    printf("%zu\\n", offsetof({struct}, {m}));\n'
    src += f'    printf("%zu\\n", sizeof({struct}));\n    return 0;\n}}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-std=c99", "-I", INCLUDE, c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    return dict(zip(members, vals[:-1])), vals[-1]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("cls,name", [("DiscosParams", "discos_params"), ("DiscosIons", "discos_ions"),
                                      ("DiscosGrid", "discos_grid"),
                                      ("DiscosReplica", "discos_replica")])
def test_ctypes_layout_matches_header(cls, name):
    st = getattr(discos, cls)
    members = [f[0] for f in st._fields_]
    offs, size = _c_layout(name, members)
    for m in members:
        assert getattr(st, m).offset == offs[m], m
    assert ctypes.sizeof(st) == size
