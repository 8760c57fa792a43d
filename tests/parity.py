"""Helpers shared by the GPU parity tests: run the HIP library and the CPU
oracle on the same model and compare their id-keyed exports bit for bit."""
from __future__ import annotations

import sys

import numpy as np

import oracle

FIELDS = ("id", "species", "x", "y", "z", "key", "event", "partner")


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32) if a.dtype == np.float32 else a


def diff_report(g: dict, o: dict) -> str:
    if len(g["id"]) != len(o["id"]):
        return f"live agents differ: gpu {len(g['id'])} oracle {len(o['id'])}"
    assert set(g) == set(o), (sorted(g), sorted(o))
    for f in FIELDS:
        if f not in g:
            continue
        ga, oa = bits(g[f]), bits(o[f])
        bad = np.nonzero(ga != oa)[0]
        if len(bad):
            k = bad[0]
            return (f"field {f}: {len(bad)} mismatches; first at id {o['id'][k]}: "
                    f"gpu {g[f][k]!r} oracle {o[f][k]!r}")
    return ""


def assert_same(g: dict, o: dict, where: str):
    msg = diff_report(g, o)
    assert not msg, f"{where}: {msg}"


def _fmix64(k: np.ndarray) -> np.ndarray:
    # MurmurHash3's 64-bit finaliser (uint64 arithmetic wraps mod 2^64)
    k = k ^ (k >> np.uint64(33))
    k = k * np.uint64(0xFF51AFD7ED558CCD)
    k = k ^ (k >> np.uint64(33))
    k = k * np.uint64(0xC4CEB9FE1A85EC53)
    return k ^ (k >> np.uint64(33))


def state_digest(e: dict) -> int:
    """The library's order-independent state digest (mabm_digest), computed
    from an id-keyed export: the sum mod 2^64 over agents of
    f(f(f((id << 32 | species) ^ c) ^ (x_bits << 32 | y_bits)) ^ z_bits)."""
    u64 = np.uint64
    ident = (e["id"].astype(u64) << u64(32)) | e["species"].astype(u64)
    xb, yb, zb = (bits(e[k]).astype(u64) for k in "xyz")
    with np.errstate(over="ignore"):
        v = _fmix64(ident ^ u64(0x9E3779B97F4A7C15))
        v = _fmix64(v ^ ((xb << u64(32)) | yb))
        v = _fmix64(v ^ zb)
        return int(v.sum(dtype=u64))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(model, checkpoints, record=True, cell_um=None, search="cells", importer=None,
             params=None):
    """Step both sides to each checkpoint and compare the full export;
    ``params`` ({parameter: value}) are set on the library's simulation."""
    import paper_2606_14603_amd as mabm
    say(f"[parity] {model.name} n={model.n_agents} checkpoints={checkpoints}")
    g = mabm.Sim(model, record=record, cell_um=cell_um)
    for k, v in (params or {}).items():
        g.set_param(k, v)
    if importer is not None:
        importer(g)
    G, _ = g.grid()
    o = oracle.OracleSim(model, grid_n=G if record else 0, search=search)
    if importer is not None:
        importer(o)
    assert_same(g.export() if record else _strip(g.export()), o.export() if record
                else _strip(o.export()), f"{model.name} t=0")
    done = 0
    for c in checkpoints:
        g.step(c - done)
        o.step(c - done)
        done = c
        ge, oe = g.export(), o.export()
        if not record:
            ge, oe = _strip(ge), _strip(oe)
        assert_same(ge, oe, f"{model.name} t={c}")
        gc, gt = g.counts()
        oc, ot = o.counts()
        assert gt == ot == c + (0 if importer is None else _t0(importer))
        assert np.array_equal(gc, oc)
    say(f"[parity] {model.name} ok, live={len(ge['id'])}")
    return g, o


def _t0(importer):
    return getattr(importer, "t0", 0)


def _strip(e: dict) -> dict:
    e = dict(e)
    for f in ("key", "event", "partner"):
        e.pop(f, None)
    return e
