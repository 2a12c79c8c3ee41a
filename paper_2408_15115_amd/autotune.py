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
        db = _load(path)
        db[key] = {k: v for k, v in res.items() if k != "cached"}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    return res
