"""CPU-side checks of the C ABI: the library builds, loads, and exports every
entry point include/sem.h declares (no compute calls: no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sem.h")).read()
    return sorted(set(re.findall(r"^\s*(?:sem_status|const char \*)\s*(sem_\w+)\s*\(", txt, re.M)))


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ["sem_mesh_create", "sem_ax", "sem_dssum", "sem_pcg_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_05640_amd import sem
    L = sem.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert sorted(sem.EXPORTED_SYMBOLS) == sorted(set(sem.EXPORTED_SYMBOLS) & set(_declared()))
    assert "gfx950" in sem.version()


def test_error_string_without_device():
    # argument validation happens before any HIP call
    import ctypes
    from paper_2405_05640_amd import sem
    h = ctypes.c_void_p()
    st = sem.lib().sem_mesh_create(None, ctypes.byref(h))
    assert st == sem.SEM_ERR_INVALID_ARG
    assert b"null" in sem.lib().sem_last_error()


def test_binding_signatures_cover_exports():
    # every exported entry point has an argtypes signature in the binding
    from paper_2405_05640_amd import sem
    L = sem.lib()
    for n in sem.EXPORTED_SYMBOLS:
        f = getattr(L, n)
        assert f.restype is not None, n
        if n not in ("sem_last_error", "sem_version"):
            assert f.argtypes is not None and len(f.argtypes) >= 1, n


def test_struct_layouts_match_header():
    # field counts of the ctypes mirrors follow the C structs in sem.h
    import re
    from paper_2405_05640_amd import sem
    txt = open(os.path.join(ROOT, "include", "sem.h")).read()

    def fields(struct_name):
        m = re.search(r"typedef struct \{([^{}]*)\}\s*%s;" % struct_name, txt)
        body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.replace("*", " ").strip()
            if not decl:
                continue
            items = decl.split(",")
            names.append(items[0].split()[-1].split("[")[0])     # "type qualifiers name"
            names += [it.strip().split("[")[0] for it in items[1:]]
        return names

    assert [f for f, _ in sem.SolveOpts._fields_] == fields("sem_solve_opts")
    assert [f for f, _ in sem.SolveReport._fields_] == fields("sem_solve_report")
    assert [f for f, _ in sem.MeshInfo._fields_] == fields("sem_mesh_info")
    assert [f for f, _ in sem.SmootherDesc._fields_] == fields("sem_smoother_desc")
