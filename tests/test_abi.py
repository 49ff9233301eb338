"""The C-ABI library loads on the CPU and exports every function declared in
include/*.h (no compute call is made here)."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sve_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for core in ("sve_init_state", "sve_step", "sve_get_state", "sve_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1307_0491_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsve.so is not built: run __graft_entry__.build()")
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(_lib.exported_symbols()) == declared_functions()


def test_package_refuses_to_run_without_device():
    import torch
    import paper_1307_0491_amd as sve
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(RuntimeError):
        sve.require_device()


def header_structs():
    """Field lists (name, C type) of the typedef'd structs in include/*.h."""
    out = {}
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        for m in re.finditer(r"typedef\s+struct\s+(\w+)\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
            fields = []
            for decl in m.group(2).split(";"):
                decl = decl.strip()
                if not decl:
                    continue
                dm = re.match(r"((?:const\s+)?\w+\s*\**)\s*(.*)", decl)
                ctype = dm.group(1).replace(" ", "")
                for name in dm.group(2).split(","):
                    name = name.strip()
                    stars = "*" * (len(name) - len(name.lstrip("*")))
                    fields.append((name.lstrip("*").strip(), ctype + stars))
            out[m.group(3)] = fields
    return out


def test_binding_structs_match_the_headers():
    """The ctypes structures have the headers' fields in the headers' order,
    with matching types (int, double, pointer)."""
    import ctypes
    from paper_1307_0491_amd import _lib
    structs = header_structs()
    pairs = {"sve_params": _lib.SveParams, "sve_bc": _lib.SveBC,
             "sve_member": _lib.SveMember}
    for cname, pyclass in pairs.items():
        assert cname in structs, cname
        want = structs[cname]
        got = pyclass._fields_
        assert [n for n, _ in want] == [n for n, _ in got], cname
        for (n, ct), (_, pt) in zip(want, got):
            if ct.endswith("*"):
                assert pt is ctypes.c_void_p, (cname, n)
            else:
                assert pt is {"int": ctypes.c_int, "double": ctypes.c_double}[ct], (cname, n)
