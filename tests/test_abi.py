"""Host-side checks of the C ABI: the library loads and exports every symbol the
header declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_2006_15234_amd", "libhpeps.so")


def declared():
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(hpeps_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared()
    for n in ("hpeps_einsumsvd_zipup", "hpeps_einsumsvd_pair", "hpeps_boundary_contract_row",
              "hpeps_peps_norm", "hpeps_peps_energy", "hpeps_apply_two_site_gate",
              "hpeps_ite_plan_create", "hpeps_ite_run"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhpeps.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2006_15234_amd import _ffi
    assert sorted(_ffi.symbols()) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhpeps.so not built")
def test_status_strings_without_gpu():
    from paper_2006_15234_amd import load_library
    lib = load_library()
    assert lib.hpeps_status_string(0) == b"ok"
    assert lib.hpeps_status_string(2) == b"shape mismatch"
    # calls with a null context fail cleanly, before touching any device
    assert lib.hpeps_destroy(None) == 1
    assert lib.hpeps_set_stream(None, None) == 1
