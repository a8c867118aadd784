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
