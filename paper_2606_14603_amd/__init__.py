"""MI355X (gfx950) molecule-agent step engine: Python binding of libmabm.so.

Argument marshalling only.  Every step of the simulation runs in the HIP
kernels of ``csrc/``; PyTorch provides the device arena (a ``torch.uint8``
tensor) and the stream.  If the library is not built, importing works but
every call raises: there is no CPU fallback.

The simulation is the per-timestep molecule-agent update of Maestri,
"Towards In Silico Cancer Therapy Design" (Abstract; Sec. 2): Brownian
motion of every molecule, proximity-based binding, product release,
compartment crossing, emission and degradation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmabm.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_CAPACITY, E_DEVICE = 0, -1, -2, -3, -4, -5
_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_STATE", -3: "E_NOMEM", -4: "E_CAPACITY",
          -5: "E_DEVICE"}
ABI_VERSION = 1
FLAG_RECORD = 1
FLAG_NO_GRAPH = 2
NONE32 = 0xFFFFFFFF
N_KERNELS = 5
PARAM_PROPOSE_LANES = 1
PARAM_PROPOSE_MIN_WORKGROUPS = 2
PARAM_BIN_EVERY_MAX = 3
PARAM_BIN_EVERY = 4
PARAM_PROPOSE_MODE = 5  # 0 auto, 1 per chunk, 2 claimer list
MAX_GRID = 1024  # cells per axis of the spatial hash, at most


class MabmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("geometry", ctypes.c_int32),
                ("box_um", ctypes.c_float), ("outer_radius_um", ctypes.c_float),
                ("inner_radius_um", ctypes.c_float), ("dt_s", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("capacity", ctypes.c_uint32),
                ("cell_um", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Rule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reactant", ctypes.c_int32 * 2),
                ("product", ctypes.c_int32 * 2), ("radius_um", ctypes.c_float),
                ("prob_per_step", ctypes.c_double), ("placement", ctypes.c_int32),
                ("release_radius_um", ctypes.c_float), ("from_comp", ctypes.c_int32),
                ("to_comp", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmabm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        c, P = ctypes, ctypes.c_void_p
        L.mabm_arena_bytes.restype = c.c_size_t
        L.mabm_arena_bytes.argtypes = [c.POINTER(Config), c.c_uint32, c.c_uint32]
        L.mabm_create_sim.argtypes = [c.POINTER(Config), P, c.c_size_t, P, c.POINTER(P)]
        L.mabm_create_sim_static.argtypes = [c.POINTER(Config), P, c.POINTER(P)]
        L.mabm_add_species.argtypes = [P, c.c_char_p, c.c_float, c.c_uint32, c.c_int32,
                                       c.POINTER(c.c_int32)]
        L.mabm_add_rule.argtypes = [P, c.POINTER(Rule), c.POINTER(c.c_int32)]
        L.mabm_grid.argtypes = [P, c.POINTER(c.c_uint32), c.POINTER(c.c_float)]
        L.mabm_step.argtypes = [P, c.c_uint32]
        L.mabm_counts.argtypes = [P, P, c.c_uint32, P]
        L.mabm_size.argtypes = [P, P, P]
        L.mabm_export.argtypes = [P, c.c_uint32, P, P, P, P, P, P, P, P]
        L.mabm_import.argtypes = [P, c.c_uint32, P, P, P, P, P, c.c_uint32, c.c_uint32]
        L.mabm_profile.argtypes = [P, c.c_int32]
        L.mabm_profile_read.argtypes = [P, P, P, P]
        L.mabm_agent_updates.argtypes = [P, P]
        L.mabm_digest.argtypes = [P, P, c.c_uint32]
        L.mabm_destroy_sim.argtypes = [P]
        L.mabm_batch_arena_bytes.restype = c.c_size_t
        L.mabm_batch_arena_bytes.argtypes = [P, c.c_uint32, c.c_uint32, c.c_uint32]
        L.mabm_create_batch.argtypes = [P, c.c_uint32, P, c.c_size_t, P, c.POINTER(P)]
        L.mabm_set_initial_counts.argtypes = [P, c.c_int32, P]
        L.mabm_batch_counts.argtypes = [P, P, c.c_uint32, P]
        L.mabm_batch_size.argtypes = [P, c.c_uint32, P, P]
        L.mabm_batch_export.argtypes = [P, c.c_uint32, c.c_uint32, P, P, P, P, P, P, P, P]
        L.mabm_batch_grid.argtypes = [P, c.c_uint32, c.POINTER(c.c_uint32), c.POINTER(c.c_float)]
        L.mabm_ring_entry_bytes.restype = c.c_size_t
        L.mabm_ring_entry_bytes.argtypes = [P]
        L.mabm_counts_ring.argtypes = [P, P, c.c_uint32, c.c_uint32]
        L.mabm_ring_read.argtypes = [P, P, c.c_uint32, P]
        L.mabm_set_param.argtypes = [P, c.c_int32, c.c_uint32]
        L.mabm_get_param.argtypes = [P, c.c_int32, P]
        L.mabm_last_error.restype = c.c_char_p
        L.mabm_last_error.argtypes = [P]
        for name in ("mabm_create_sim", "mabm_create_sim_static", "mabm_add_species", "mabm_add_rule", "mabm_grid",
                     "mabm_step", "mabm_counts", "mabm_size", "mabm_export", "mabm_import",
                     "mabm_profile", "mabm_profile_read", "mabm_agent_updates", "mabm_digest",
                     "mabm_destroy_sim", "mabm_create_batch", "mabm_set_initial_counts",
                     "mabm_batch_counts", "mabm_batch_size", "mabm_batch_export",
                     "mabm_batch_grid", "mabm_counts_ring", "mabm_ring_read",
                     "mabm_set_param", "mabm_get_param"):
            getattr(L, name).restype = c.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_config(model, record: bool = False, cell_um: Optional[float] = None,
                capacity: Optional[int] = None, graphs: bool = False) -> Config:
    flags = (FLAG_RECORD if record else 0) | (0 if graphs else FLAG_NO_GRAPH)
    return Config(ABI_VERSION, int(model.geometry), float(model.box_um),
                  float(model.outer_radius_um), float(model.inner_radius_um), float(model.dt_s),
                  int(model.seed), int(capacity if capacity is not None else model.capacity),
                  float(cell_um if cell_um is not None else model.cell_um), flags)


def arena_bytes(model, record: bool = False, cell_um: Optional[float] = None,
                capacity: Optional[int] = None) -> int:
    cfg = make_config(model, record, cell_um, capacity)
    return int(lib().mabm_arena_bytes(ctypes.byref(cfg), len(model.species), len(model.rules)))


class Sim:
    """One simulation on the GPU.  ``model`` is a workloads.Model (species,
    rules, geometry, dt, seed, capacity).  By default the simulation gets its
    own HIP stream; ``graphs=True`` replays each step as a captured HIP graph
    (measured slightly slower than direct launches on ROCm 7.2).
    ``static_arena=True`` creates it in the library's static device arena
    (mabm_create_sim_static, for callers that cannot allocate): no arena
    tensor is allocated, and steps are direct launches."""

    def __init__(self, model, record: bool = False, cell_um: Optional[float] = None,
                 capacity: Optional[int] = None, stream=None, device: str = "cuda",
                 arena=None, graphs: bool = False, static_arena: bool = False):
        import torch
        L = lib()
        self.n_species = len(model.species)
        self.cfg = make_config(model, record, cell_um, capacity, graphs)
        nbytes = int(L.mabm_arena_bytes(ctypes.byref(self.cfg), self.n_species,
                                        len(model.rules)))
        if nbytes == 0:
            raise MabmError(E_INVALID, "invalid configuration")
        if static_arena:
            self.arena = None
            dev = torch.device(device)
        else:
            self.arena = arena if arena is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                                      device=device)
            dev = self.arena.device
        if stream is None:
            stream = torch.cuda.Stream(dev)
            stream.wait_stream(torch.cuda.current_stream(dev))
        self.stream = stream
        self.device = dev
        h = ctypes.c_void_p()
        if static_arena:
            rc = L.mabm_create_sim_static(ctypes.byref(self.cfg),
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        else:
            rc = L.mabm_create_sim(ctypes.byref(self.cfg), ctypes.c_void_p(self.arena.data_ptr()),
                                   self.arena.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h))
        if rc != OK:
            raise MabmError(rc, L.mabm_last_error(None).decode())
        self._h = h
        self._lib = L
        self._add_model(model)

    def _add_model(self, model):
        L, h = lib(), self._h
        out = ctypes.c_int32()
        for sp in model.species:
            self._chk(L.mabm_add_species(h, sp.name.encode(), float(sp.diffusion_um2_s),
                                         int(sp.count), int(sp.compartment), ctypes.byref(out)))
        for r in model.rules:
            rr = Rule(int(r.kind), (ctypes.c_int32 * 2)(*r.reactants),
                      (ctypes.c_int32 * 2)(*r.products), float(r.radius_um),
                      float(r.prob_per_step), int(r.placement), float(r.release_radius_um),
                      int(r.from_comp), int(r.to_comp))
            self._chk(L.mabm_add_rule(h, ctypes.byref(rr), ctypes.byref(out)))

    def _chk(self, rc: int) -> int:
        if rc != OK:
            raise MabmError(rc, lib().mabm_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            # the library handle is held by the object, so that a simulation
            # collected at interpreter exit can still be destroyed
            self._lib.mabm_destroy_sim(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        self._chk(lib().mabm_step(self._h, int(n)))

    def grid(self):
        g = ctypes.c_uint32()
        h = ctypes.c_float()
        self._chk(lib().mabm_grid(self._h, ctypes.byref(g), ctypes.byref(h)))
        return int(g.value), float(h.value)

    def counts(self):
        out = np.zeros(self.n_species, np.uint64)
        t = np.zeros(1, np.uint64)
        self._chk(lib().mabm_counts(self._h, _ptr(out), self.n_species, _ptr(t)))
        return out, int(t[0])

    def size(self):
        n = np.zeros(1, np.uint32)
        nid = np.zeros(1, np.uint32)
        self._chk(lib().mabm_size(self._h, _ptr(n), _ptr(nid)))
        return int(n[0]), int(nid[0])

    def export(self) -> dict:
        n, _ = self.size()
        m = max(n, 1)
        out = dict(id=np.zeros(m, np.uint32), species=np.zeros(m, np.uint8),
                   x=np.zeros(m, np.float32), y=np.zeros(m, np.float32),
                   z=np.zeros(m, np.float32), key=np.zeros(m, np.uint32),
                   event=np.zeros(m, np.int32), partner=np.zeros(m, np.uint32))
        self._chk(lib().mabm_export(self._h, m, *(_ptr(out[k]) for k in
                                                 ("id", "species", "x", "y", "z", "key", "event",
                                                  "partner"))))
        return {k: v[:n] for k, v in out.items()}

    def import_state(self, ids, species, x, y, z, next_id: int, t: int = 0):
        ids = np.ascontiguousarray(ids, np.uint32)
        species = np.ascontiguousarray(species, np.uint8)
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        z = np.ascontiguousarray(z, np.float32)
        self._chk(lib().mabm_import(self._h, len(ids), _ptr(ids), _ptr(species), _ptr(x),
                                    _ptr(y), _ptr(z), int(next_id), int(t)))

    def profile(self, enable: bool = True):
        self._chk(lib().mabm_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        names = (ctypes.c_char_p * N_KERNELS)()
        launches = np.zeros(N_KERNELS, np.uint64)
        ms = np.zeros(N_KERNELS, np.float64)
        self._chk(lib().mabm_profile_read(self._h, ctypes.cast(names, ctypes.c_void_p),
                                          _ptr(launches), _ptr(ms)))
        return {(names[k] or b"kernel%d" % k).decode(): (int(launches[k]), float(ms[k]))
                for k in range(N_KERNELS)}

    def set_param(self, param: int, value: int):
        """Performance parameter (PARAM_PROPOSE_LANES, PARAM_PROPOSE_MIN_WORKGROUPS,
        PARAM_BIN_EVERY_MAX, PARAM_PROPOSE_MODE); results do not depend on them."""
        self._chk(lib().mabm_set_param(self._h, int(param), int(value)))

    def get_param(self, param: int) -> int:
        """A parameter's value; PARAM_BIN_EVERY gives the steps between
        binnings in effect."""
        v = ctypes.c_uint32()
        self._chk(lib().mabm_get_param(self._h, int(param), ctypes.byref(v)))
        return int(v.value)

    def record_counts(self, every: int, entries: int = 4096):
        """Append the live counts to a device ring every ``every`` steps
        (0 stops); the ring holds the newest ``entries`` entries."""
        import torch
        L = lib()
        if every <= 0:
            # the library synchronises the simulation's stream before it lets
            # go of the old ring, so the buffer is free once this returns
            self._chk(L.mabm_counts_ring(self._h, None, 0, 0))
            self._ring = None
            return
        words = int(L.mabm_ring_entry_bytes(self._h)) // 8
        dev = self.device
        ring = torch.zeros(entries * words, dtype=torch.int64, device=dev)
        # the zero fill runs on the current stream: the simulation's stream,
        # which writes the entries, waits for it, and the caching allocator
        # is told that the buffer is in use on that stream
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        ring.record_stream(self.stream)
        self._chk(L.mabm_counts_ring(self._h, ctypes.c_void_p(ring.data_ptr()), entries,
                                     int(every)))
        self._ring = ring
        self._ring_words, self._ring_entries = words, entries

    def ring(self):
        """(steps, counts): the recorded entries, oldest first; counts has
        shape (entries, simulations, species)."""
        n = np.zeros(1, np.uint64)
        buf = np.zeros(self._ring_entries * self._ring_words, np.uint64)
        self._chk(lib().mabm_ring_read(self._h, _ptr(buf), self._ring_entries, _ptr(n)))
        m = int(min(n[0], self._ring_entries))
        e = buf[:m * self._ring_words].reshape(m, self._ring_words)
        sims = (self._ring_words - 1) // 64
        return e[:, 0].copy(), e[:, 1:].reshape(m, sims, 64)[:, :, :self.n_species].copy()

    def agent_updates(self) -> int:
        out = np.zeros(1, np.uint64)
        self._chk(lib().mabm_agent_updates(self._h, _ptr(out)))
        return int(out[0])

    def digest(self) -> np.ndarray:
        """Order-independent 64-bit digest of the id-keyed state, one per
        simulation of the handle (uint64 array)."""
        n = getattr(self, "n_sims", 1)
        out = np.zeros(n, np.uint64)
        self._chk(lib().mabm_digest(self._h, _ptr(out), n))
        return out


def _same_structure(a, b) -> bool:
    sa = [(x.name, float(x.diffusion_um2_s), int(x.compartment)) for x in a.species]
    sb = [(x.name, float(x.diffusion_um2_s), int(x.compartment)) for x in b.species]
    return (sa == sb and list(a.rules) == list(b.rules) and a.geometry == b.geometry
            and a.dt_s == b.dt_s)


def batch_arena_bytes(models, record: bool = False) -> int:
    cfgs = (Config * len(models))(*[make_config(m, record) for m in models])
    return int(lib().mabm_batch_arena_bytes(ctypes.cast(cfgs, ctypes.c_void_p), len(models),
                                            len(models[0].species), len(models[0].rules)))


class Batch(Sim):
    """Many simulations of one model (same species, rules, geometry and dt)
    stepped together by one set of launches per step; each keeps its own
    seed, volume, capacity and initial counts (``models[k]`` for simulation
    k), and its trajectory is the one ``Sim(models[k])`` gives."""

    def __init__(self, models, record: bool = False, stream=None, device: str = "cuda",
                 arena=None, graphs: bool = False):
        import torch
        L = lib()
        if not models:
            raise MabmError(E_INVALID, "empty batch")
        m0 = models[0]
        for m in models[1:]:
            if not _same_structure(m0, m):
                raise MabmError(E_INVALID, f"{m.name}: a batch shares species, rules, geometry, dt")
        self.n_sims = len(models)
        self.n_species = len(m0.species)
        self.cfgs = (Config * self.n_sims)(*[make_config(m, record, None, None, graphs)
                                             for m in models])
        nbytes = int(L.mabm_batch_arena_bytes(ctypes.cast(self.cfgs, ctypes.c_void_p),
                                              self.n_sims, self.n_species, len(m0.rules)))
        if nbytes == 0:
            raise MabmError(E_INVALID, "invalid batch configuration")
        self.arena = arena if arena is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                                  device=device)
        if stream is None:
            stream = torch.cuda.Stream(self.arena.device)
            stream.wait_stream(torch.cuda.current_stream(self.arena.device))
        self.stream = stream
        self.device = self.arena.device
        h = ctypes.c_void_p()
        rc = L.mabm_create_batch(ctypes.cast(self.cfgs, ctypes.c_void_p), self.n_sims,
                                 ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise MabmError(rc, L.mabm_last_error(None).decode())
        self._h = h
        self._lib = L
        self._add_model(m0)
        for k in range(self.n_species):
            c = np.array([int(m.species[k].count) for m in models], np.uint32)
            self._chk(L.mabm_set_initial_counts(h, k, _ptr(c)))

    def counts(self):
        """(n_sims, n_species) live counts and the step counter."""
        out = np.zeros(self.n_sims * self.n_species, np.uint64)
        t = np.zeros(1, np.uint64)
        self._chk(lib().mabm_batch_counts(self._h, _ptr(out), self.n_species, _ptr(t)))
        return out.reshape(self.n_sims, self.n_species), int(t[0])

    def size(self, k: int = 0):
        n = np.zeros(1, np.uint32)
        nid = np.zeros(1, np.uint32)
        self._chk(lib().mabm_batch_size(self._h, int(k), _ptr(n), _ptr(nid)))
        return int(n[0]), int(nid[0])

    def grid(self, k: int = 0):
        g = ctypes.c_uint32()
        h = ctypes.c_float()
        self._chk(lib().mabm_batch_grid(self._h, int(k), ctypes.byref(g), ctypes.byref(h)))
        return int(g.value), float(h.value)

    def export(self, k: int = 0) -> dict:
        n, _ = self.size(k)
        m = max(n, 1)
        out = dict(id=np.zeros(m, np.uint32), species=np.zeros(m, np.uint8),
                   x=np.zeros(m, np.float32), y=np.zeros(m, np.float32),
                   z=np.zeros(m, np.float32), key=np.zeros(m, np.uint32),
                   event=np.zeros(m, np.int32), partner=np.zeros(m, np.uint32))
        self._chk(lib().mabm_batch_export(self._h, int(k), m,
                                          *(_ptr(out[f]) for f in
                                            ("id", "species", "x", "y", "z", "key", "event",
                                             "partner"))))
        return {f: v[:n] for f, v in out.items()}

    def import_state(self, *a, **kw):
        raise MabmError(E_STATE, "a batch cannot import a state")
