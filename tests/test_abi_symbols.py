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


def test_grid_limit_and_cell_total(lib):
    # a 1,024-cell grid per axis is the largest; the cell grids of one handle
    # hold at most 2^31 cells together (32-bit cell keys and prefix sums)
    import paper_2606_14603_amd as mabm
    import workloads as W
    L = mabm.lib()
    assert mabm.MAX_GRID == 1024
    m = W.c2(20_000, seed=9).with_(outer_radius_um=5.4, cell_um=0.01054)
    ns, nr = len(m.species), len(m.rules)

    def arena(model):
        c = mabm.make_config(model)
        return L.mabm_arena_bytes(ctypes.byref(c), ns, nr)

    one = arena(m)
    assert one > 12 * (1 << 30)  # cell counts, starts and chain heads of 2^30 cells
    assert arena(m.with_(cell_um=0.0211)) < one // 6  # 511 cells per axis
    assert arena(m.with_(cell_um=0.001)) == one  # coarsened to 1,024
    c = mabm.make_config(m)
    arr = (type(c) * 3)(c, c, c)
    fn = L.mabm_batch_arena_bytes
    fn.restype = ctypes.c_size_t
    assert fn(arr, 2, ns, nr) > 2 * 12 * (1 << 30)
    assert fn(arr, 3, ns, nr) == 0
    h = ctypes.c_void_p()
    rc = L.mabm_create_batch(ctypes.cast(arr, ctypes.c_void_p), 3, None, 0, None, ctypes.byref(h))
    assert rc == mabm.E_INVALID and not h.value
    assert b"2^31 cells" in L.mabm_last_error(None)
