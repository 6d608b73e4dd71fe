"""The C-ABI library loads and exports every entry point declared in include/*.h
(CPU only: nothing is called that needs a GPU)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2204_14167_amd import discos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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
                     "discos_interpolate", "discos_near_field", "discos_step", "discos_check",
                     "discos_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(discos.LIB_PATH):
        pytest.fail("libdiscos.so not built (python -m paper_2204_14167_amd.build)")
    lib = ctypes.CDLL(discos.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_ctypes_layout_matches_header():
    # offsets of the struct members as the C compiler lays them out on x86-64
    expect = dict(eps=0, bc_type=8, bc_value=16, e_ext=32, psi=56, p3m_table=64, p3m_len=72,
                  p3m_dr=80, wall_on=88, wall_sigma=96, lj_on=120, lj_range=152, kT=160,
                  nspecies=184, radius=192, mob_coef=200, seed=208)
    for k, v in expect.items():
        assert getattr(discos.DiscosParams, k).offset == v, k
    assert ctypes.sizeof(discos.DiscosParams) == 216
    assert ctypes.sizeof(discos.DiscosIons) == 40
