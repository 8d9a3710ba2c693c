"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects invalid configurations before touching
a device."""
import ctypes as ct
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.environ.get("CELLFFT_LIBRARY") or os.path.join(ROOT, "paper_2004_05197_amd", "libcellfft.so")


@pytest.fixture(scope="module")
def cdll():
    if not os.path.exists(LIB):
        from paper_2004_05197_amd import build
        build.build()
    return ct.CDLL(LIB)


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s+(cell_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["cell_create", "cell_set_material", "cell_solve", "cell_effective_stiffness",
                     "cell_adjoint", "cell_get_displacement", "cell_destroy", "cell_last_error"]:
        assert required in names


def test_every_declared_symbol_is_exported(cdll):
    missing = [n for n in declared_functions() if not hasattr(cdll, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2004_05197_amd import binding
    assert set(declared_functions()) == set(binding.exported_symbols())


def test_invalid_configs_rejected_without_a_device():
    from paper_2004_05197_amd import binding as B
    with pytest.raises(B.CellError) as e:
        B.Cell((10, 8, 8))
    assert e.value.status == B.CELL_E_UNSUPPORTED
    with pytest.raises(B.CellError) as e:
        B.Cell((8, 8, 8), precision=7)
    assert e.value.status == B.CELL_E_ARG
    with pytest.raises(B.CellError) as e:
        B.Cell((8, 8, 8), max_loads=9)
    assert e.value.status == B.CELL_E_ARG
    with pytest.raises(B.CellError) as e:
        B.Cell((8, 8, 8, 8))
    assert e.value.status == B.CELL_E_ARG
    assert "dim" in B.last_error()


def test_null_arguments(cdll):
    cdll.cell_create.restype = ct.c_int
    assert cdll.cell_create(None, None) == -1
    cdll.cell_last_error.restype = ct.c_char_p
    assert b"null" in cdll.cell_last_error()


def test_normal_build_checks_no_bounds(cdll):
    # the bounds counter exists only in the checked build; the normal one
    # answers -1 without touching a device
    cdll.cell_debug_bounds_violations.restype = ct.c_int
    assert cdll.cell_debug_bounds_violations() == -1


def test_last_error_is_per_thread():
    # argument validation fails before any device work, so two threads can
    # each see their own message
    import threading
    from paper_2004_05197_amd import binding as B
    msgs = {}

    def fail_here():
        with pytest.raises(B.CellError):
            B.Cell((10, 8, 8))
        msgs["other"] = B.last_error()

    with pytest.raises(B.CellError):
        B.Cell((8, 8, 8), precision=7)
    mine = B.last_error()
    t = threading.Thread(target=fail_here)
    t.start()
    t.join()
    assert "grid size 10" in msgs["other"]
    assert mine == "invalid precision" and B.last_error() == mine
