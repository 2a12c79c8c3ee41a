"""Autotuner of the lattice kernel's launch schedule for a set of cases.

It times candidate schedules (threads per tile, tile schedule, persistent
workgroup count, tile order) of the fused stream + collide kernel on a
fluid-only context over the same boxes (the kernel's run time does not depend
on the population values, and the results are bitwise independent of the
schedule), keeps the fastest, and caches it in a JSON file keyed by GPU
architecture, storage and the case mix.  Every timing runs the library's own
kernel through the C ABI; this module only orchestrates.
"""
from __future__ import annotations

import hashlib
import json
import os

CACHE_ENV = "TURRET_AUTOTUNE_CACHE"


def default_candidates(n_cu=256):
    c = [dict(block=256, schedule=0, persist_wgs=0, tile_order=0),
         dict(block=128, schedule=0, persist_wgs=0, tile_order=0),
         dict(block=256, schedule=1, persist_wgs=0, tile_order=0)]
    for wgs in (4 * n_cu, 8 * n_cu, 16 * n_cu):
        c.append(dict(block=256, schedule=2, persist_wgs=wgs, tile_order=1))
        c.append(dict(block=256, schedule=3, persist_wgs=wgs, tile_order=2))
        c.append(dict(block=256, schedule=4, persist_wgs=wgs, tile_order=2))
        c.append(dict(block=256, schedule=4, persist_wgs=wgs, tile_order=0))
    c.append(dict(block=128, schedule=3, persist_wgs=16 * n_cu, tile_order=2))
    return c


def cache_path():
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "turret", "autotune.json"))


def cache_key(arch, storage, cases):
    desc = [arch, storage, [(c["nx"], c["ny"], c["nz"], c.get("bc_zlo", 0), c.get("bc_zhi", 0),
                             c.get("sponge", 0)) for c in cases]]
    return hashlib.sha1(json.dumps(desc).encode()).hexdigest()[:20]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(cases, storage="f32", candidates=None, launches=8, warmup=2, use_cache=True, path=None):
    """Return {"best": options, "ms": best ms per launch, "table": [...],
    "key": cache key, "cached": bool}."""
    import torch

    from . import turret as T

    path = path or cache_path()
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name)
    key = cache_key(arch, storage, cases)
    db = _load(path) if use_cache else {}
    if key in db:
        hit = dict(db[key])
        hit["cached"] = True
        return hit
    cands = candidates or default_candidates(props.multi_processor_count)
    stream = torch.cuda.Stream()
    S = T.Solver(cases, None, storage=storage, stream=stream)
    table = []
    for cand in cands:
        S.set_schedule(**cand)
        for _ in range(warmup):
            S.lbm_step()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(launches):
            S.lbm_step()
        b.record(stream)
        torch.cuda.synchronize()
        table.append({"options": cand, "ms": a.elapsed_time(b) / launches})
    S.close()
    del S
    torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    res = {"best": best["options"], "ms": best["ms"], "table": table, "key": key, "arch": arch,
           "storage": storage, "cached": False}
    if use_cache:
        _store(path, key, res)
    return res


def _store(path, key, res):
    db = _load(path)
    db[key] = {k: v for k, v in res.items() if k != "cached"}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, path)


def tune_step(cases, bodies, storage="f32", top=3, steps=12, warmup=3, use_cache=True, path=None, candidates=None):
    """Schedule for the whole coupled step rather than the lattice kernel
    alone: the coupling can run on the library's second stream beside the
    lattice kernel, and a schedule that leaves room on the CUs can hide it
    (how much it hides also depends on the runtime giving the two streams
    different hardware queues).  Times full steps (body advance, lattice
    kernel, coupling, window) for the `top` fastest lattice-kernel schedules
    of tune() and the fastest persistent one with the coupling beside, and
    the fastest schedule with the coupling after the lattice kernel
    (serial_ibm), and keeps the fastest step.  Returns {"best" (schedule and
    serial_ibm), "ms" (per step), "lattice_ms" (the lattice kernel alone
    under that schedule), "table", "key", "cached"}."""
    import torch

    from . import turret as T

    path = path or cache_path()
    lat = tune(cases, storage=storage, candidates=candidates, use_cache=use_cache, path=path)
    key = lat["key"] + "-step-" + hashlib.sha1(
        json.dumps([int(b["x_body"].shape[0]) if b is not None else 0 for b in bodies]).encode()).hexdigest()[:8]
    db = _load(path) if use_cache else {}
    if key in db:
        hit = dict(db[key])
        hit["cached"] = True
        return hit
    ranked = sorted(lat["table"], key=lambda r: r["ms"])
    picks = [r["options"] for r in ranked[:top]]
    persistent = [r["options"] for r in ranked if r["options"]["schedule"] >= 2]
    if persistent and persistent[0] not in picks:
        picks.append(persistent[0])
    lat_ms = {json.dumps(r["options"], sort_keys=True): r["ms"] for r in ranked}
    # each schedule with the coupling beside the lattice kernel, and the
    # fastest lattice schedule with the coupling after it on one stream
    picks = [dict(c, serial_ibm=0) for c in picks] + [dict(picks[0], serial_ibm=1)]
    table = []
    for cand in picks:
        stream = torch.cuda.Stream()
        S = T.Solver(cases, bodies, storage=storage, stream=stream, **cand)
        S.run(warmup)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        S.run(steps)
        b.record(stream)
        torch.cuda.synchronize()
        sched = {k: v for k, v in cand.items() if k != "serial_ibm"}
        table.append({"options": cand, "ms": a.elapsed_time(b) / steps,
                      "lattice_ms": lat_ms[json.dumps(sched, sort_keys=True)]})
        S.close()
        del S
        torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    res = {"best": best["options"], "ms": best["ms"], "lattice_ms": best["lattice_ms"], "table": table,
           "key": key, "storage": storage, "cached": False}
    if use_cache:
        _store(path, key, res)
    return res
