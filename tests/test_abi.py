"""The C ABI library loads and exports every function include/sadmm.h declares
(no device needed: nothing is called)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sadmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sadmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2307_08606_amd", "libsadmm.so"))
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_abi():
    from paper_2307_08606_amd import sadmm_lib
    assert set(declared_functions()) <= set(sadmm_lib.EXPORTED)


def test_params_struct_layout_matches_header():
    """The ctypes mirror of sadmm_params has the header's field order."""
    from paper_2307_08606_amd import sadmm_lib
    src = open(os.path.join(ROOT, "include", "sadmm.h")).read()
    body = src[src.index("typedef struct {", src.index("sadmm_storage;")):src.index("} sadmm_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.replace("typedef struct {", "").strip()
        if not decl:
            continue
        parts = decl.split(None, 1)
        for v in parts[1].split(","):
            names.append(v.strip().lstrip("*"))
    got = [f[0].rstrip("_") for f in sadmm_lib.sadmm_params._fields_]
    assert got == names
