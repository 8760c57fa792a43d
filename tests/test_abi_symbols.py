"""CPU checks of the C ABI: the built library loads and exports every
function that include/mabm.h declares; host-only calls (footprint,
configuration validation) behave as documented.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mabm.h")
LIB = os.path.join(ROOT, "paper_2606_14603_amd", "libmabm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mabm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmabm.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_verbs():
    names = declared()
    for verb in ("mabm_create_sim", "mabm_add_species", "mabm_add_rule", "mabm_step",
                 "mabm_counts", "mabm_export", "mabm_import", "mabm_destroy_sim",
                 "mabm_arena_bytes", "mabm_last_error"):
        assert verb in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_arena_bytes_and_config_validation(lib):
    import paper_2606_14603_amd as mabm
    import workloads as W
    m = W.c2()
    b = mabm.arena_bytes(m)
    # two agent buffers of 17 B plus per-agent scratch, per capacity slot
    assert b > 2 * 17 * m.capacity
    assert b < 200 * m.capacity
    bad = mabm.make_config(m)
    bad.dt_s = 0.0
    assert lib.mabm_arena_bytes(ctypes.byref(bad), 8, 12) == 0
    h = ctypes.c_void_p()
    L = mabm.lib()
    rc = L.mabm_create_sim(ctypes.byref(bad), None, 0, None, ctypes.byref(h))
    assert rc == mabm.E_INVALID and not h.value
    assert b"dt_s" in L.mabm_last_error(None)
