"""ctypes binding of the plain-C CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(``paper_2606_14603_amd``) never does, and this package never imports it.

The oracle computes the molecule-agent step of the paper (Abstract; Sec. 2)
under the step definition O0..O10 (stated phase by phase in mabm_oracle.c),
literally and slowly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "mabm_oracle.c")

# gcc flags: IEEE binary32 evaluated as written (no contraction, no
# reassociation); plain -O2, no vector ISA beyond the x86-64 baseline;
# OpenMP for the two per-agent loops whose iterations are independent.
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wextra"]

E_CODES = {0: "OK", -1: "E_INVALID", -2: "E_STATE", -3: "E_NOMEM", -4: "E_CAPACITY",
           -5: "E_DEVICE"}
NONE32 = 0xFFFFFFFF


def build(out: str = LIB_PATH) -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC_PATH, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, out)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        L.orc_create.restype = c.c_void_p
        L.orc_create.argtypes = [c.c_int, c.c_float, c.c_float, c.c_float, c.c_float,
                                 c.c_uint64, c.c_uint32, c.c_uint32]
        L.orc_destroy.argtypes = [c.c_void_p]
        L.orc_last_error.restype = c.c_char_p
        L.orc_last_error.argtypes = [c.c_void_p]
        L.orc_add_species.argtypes = [c.c_void_p, c.c_float, c.c_uint32, c.c_int]
        L.orc_add_rule.argtypes = [c.c_void_p, c.c_int, c.c_int, c.c_int, c.c_int, c.c_int,
                                   c.c_float, c.c_double, c.c_int, c.c_float, c.c_int, c.c_int]
        L.orc_set_search.argtypes = [c.c_void_p, c.c_int]
        P = c.c_void_p
        L.orc_import.argtypes = [c.c_void_p, c.c_uint32, P, P, P, P, P, c.c_uint32, c.c_uint32]
        L.orc_step.argtypes = [c.c_void_p, c.c_uint32]
        L.orc_counts.argtypes = [c.c_void_p, P, c.c_uint32, P]
        L.orc_size.argtypes = [c.c_void_p, P, P]
        L.orc_export.argtypes = [c.c_void_p, c.c_uint32, P, P, P, P, P, P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_log.restype = c.c_float
        L.orc_log.argtypes = [c.c_float]
        L.orc_sincos2pi.argtypes = [c.c_float, P, P]
        L.orc_gauss3.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, P]
        L.orc_event_word.restype = c.c_uint32
        L.orc_event_word.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32]
        L.orc_threads.restype = c.c_int
        L.orc_threads.argtypes = [c.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{E_CODES.get(code, code)}: {msg}")
        self.code = code


class OracleSim:
    """One simulation held by the oracle.  ``model`` is a workloads.Model."""

    def __init__(self, model, grid_n: int = 0, search: str = "cells", capacity: int | None = None):
        L = lib()
        cap = capacity if capacity is not None else model.capacity
        h = L.orc_create(int(model.geometry), float(model.box_um), float(model.outer_radius_um),
                         float(model.inner_radius_um), float(model.dt_s), int(model.seed),
                         int(cap), int(grid_n))
        if not h:
            raise OracleError(-1, "invalid configuration")
        self._h = h
        self.n_species = len(model.species)
        for sp in model.species:
            self._chk(L.orc_add_species(h, float(sp.diffusion_um2_s), int(sp.count),
                                        int(sp.compartment)))
        for r in model.rules:
            self._chk(L.orc_add_rule(h, int(r.kind), int(r.reactants[0]), int(r.reactants[1]),
                                     int(r.products[0]), int(r.products[1]), float(r.radius_um),
                                     float(r.prob_per_step), int(r.placement),
                                     float(r.release_radius_um), int(r.from_comp),
                                     int(r.to_comp)))
        if search not in ("cells", "brute"):
            raise ValueError(search)
        self._chk(L.orc_set_search(h, 0 if search == "cells" else 1))

    def _chk(self, rc: int) -> int:
        if rc < 0:
            raise OracleError(rc, lib().orc_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        self._chk(lib().orc_step(self._h, int(n)))

    def counts(self):
        out = np.zeros(self.n_species, np.uint64)
        t = np.zeros(1, np.uint64)
        self._chk(lib().orc_counts(self._h, _ptr(out), self.n_species, _ptr(t)))
        return out, int(t[0])

    def size(self):
        n = np.zeros(1, np.uint32)
        nid = np.zeros(1, np.uint32)
        self._chk(lib().orc_size(self._h, _ptr(n), _ptr(nid)))
        return int(n[0]), int(nid[0])

    def export(self) -> dict:
        n, _ = self.size()
        m = max(n, 1)
        out = dict(id=np.zeros(m, np.uint32), species=np.zeros(m, np.uint8),
                   x=np.zeros(m, np.float32), y=np.zeros(m, np.float32),
                   z=np.zeros(m, np.float32), key=np.zeros(m, np.uint32),
                   event=np.zeros(m, np.int32), partner=np.zeros(m, np.uint32))
        self._chk(lib().orc_export(self._h, m, *(_ptr(out[k]) for k in
                                                ("id", "species", "x", "y", "z", "key", "event",
                                                 "partner"))))
        return {k: v[:n] for k, v in out.items()}

    def import_state(self, ids, species, x, y, z, next_id: int, t: int = 0):
        ids = np.ascontiguousarray(ids, np.uint32)
        species = np.ascontiguousarray(species, np.uint8)
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        z = np.ascontiguousarray(z, np.float32)
        self._chk(lib().orc_import(self._h, len(ids), _ptr(ids), _ptr(species), _ptr(x), _ptr(y),
                                   _ptr(z), int(next_id), int(t)))


# ---- building blocks, for the pin tests ----

def threads(n: int = 0) -> int:
    """Threads of the oracle's parallel per-agent loops (n > 0 sets them);
    returns the count the next step uses."""
    return int(lib().orc_threads(int(n)))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def log(x: float) -> float:
    return lib().orc_log(float(x))


def sincos2pi(a: float):
    s = np.zeros(1, np.float32)
    c = np.zeros(1, np.float32)
    lib().orc_sincos2pi(float(a), _ptr(s), _ptr(c))
    return float(s[0]), float(c[0])


def event_word(seed: int, agent_id: int, t: int) -> int:
    return int(lib().orc_event_word(int(seed), int(agent_id), int(t)))


def gauss3(seed: int, agent_id: int, t: int) -> np.ndarray:
    out = np.zeros(3, np.float32)
    lib().orc_gauss3(int(seed), int(agent_id), int(t), _ptr(out))
    return out
