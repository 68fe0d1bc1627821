"""Autotuner for the AxLocal launch shape on gfx950.

For each (order N, geometry kind, precision) it times the kernel with the default and the
alternative elements-per-work-group shape and several persistent grid sizes on a synthetic mesh
of about 2^22 local nodes, keeps the fastest, and writes a JSON cache.  ``load()`` pushes a
cache into the library (``ax_tune_set``); the package calls it on import when the cache for this
architecture exists.  Tuning never changes results, only the launch shape.

    python -m paper_2504_07042_amd.autotune            # tune everything, write the cache
    python -m paper_2504_07042_amd.autotune --N 7      # one order
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import time

import numpy as np

from . import AX_FP32, AX_FP64, AX_PARALLELEPIPED, AX_STORED_G, AX_TRILINEAR, Basis, _check, lib

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
GEOMS = {"trilinear": AX_TRILINEAR, "parallelepiped": AX_PARALLELEPIPED, "stored": AX_STORED_G}
PRECS = {"fp64": AX_FP64, "fp32": AX_FP32}
GRID_MULTS = (1, 2, 4, 8)


def tune_get(N: int, geom: int, prec: int):
    a, g, e = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().ax_tune_get(N, geom, prec, ctypes.byref(a), ctypes.byref(g), ctypes.byref(e)))
    return {"epb_alt": a.value, "grid_mult": g.value, "elems_per_group": e.value}


def tune_set(N: int, geom: int, prec: int, epb_alt: int, grid_mult: int):
    _check(lib().ax_tune_set(N, geom, prec, int(epb_alt), int(grid_mult)))


def load(path: str = CACHE) -> int:
    """Apply a tuning cache; returns the number of entries applied (0 if there is none)."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for ent in data.get("entries", []):
        tune_set(ent["N"], GEOMS[ent["geom"]], PRECS[ent["prec"]], ent["epb_alt"], ent["grid_mult"])
        n += 1
    return n


def _time(fn, reps=20, warmup=3):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def tune(orders=range(1, 16), geoms=tuple(GEOMS), precs=tuple(PRECS), target_nodes=1 << 22, verbose=True):
    import torch
    from . import ax_local, ax_local_precomputedG, geom_factors, meshgen, parallelepiped_factors
    entries = []
    for N in orders:
        b = Basis(N)
        grid = meshgen.grid_for_nodes(N, target_nodes)
        m = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
        pm, _ = meshgen.parallelepiped_hex(*grid, seed=2)
        V = torch.from_numpy(m.verts).cuda()
        h = parallelepiped_factors(torch.from_numpy(pm.verts).cuda())
        X64 = torch.from_numpy(meshgen.random_nodal(m.E, N, seed=N)).cuda()
        for pname in precs:
            prec = PRECS[pname]
            X = X64 if prec == AX_FP64 else X64.float()
            Y = torch.empty_like(X)
            G = None
            for gname in geoms:
                geom = GEOMS[gname]
                if geom == AX_STORED_G:
                    G, _ = geom_factors(V, b, prec)
                    fn = lambda: ax_local_precomputedG(X, G, b, prec, out=Y)
                elif geom == AX_TRILINEAR:
                    fn = lambda: ax_local(X, V, b, AX_TRILINEAR, prec, out=Y)
                else:
                    fn = lambda: ax_local(X, h, b, AX_PARALLELEPIPED, prec, out=Y)
                best = None
                alts = (0, 1) if tune_get(N, geom, prec)["elems_per_group"] != _elems(N, geom, prec, 1) else (0,)
                for alt in alts:
                    for gm in GRID_MULTS:
                        tune_set(N, geom, prec, alt, gm)
                        t = _time(fn)
                        if best is None or t < best[0]:
                            best = (t, alt, gm)
                tune_set(N, geom, prec, best[1], best[2])
                ent = {"N": N, "geom": gname, "prec": pname, "epb_alt": best[1], "grid_mult": best[2],
                       "elems_per_group": tune_get(N, geom, prec)["elems_per_group"],
                       "GDOFs": round(m.E * (N + 1) ** 3 / best[0] / 1e9, 2)}
                entries.append(ent)
                if verbose:
                    print(json.dumps(ent), flush=True)
                del fn
            del G
    return {"arch": "gfx950", "target_nodes": target_nodes, "created": time.strftime("%Y-%m-%d"),
            "entries": entries}


def _elems(N, geom, prec, alt):
    cur = tune_get(N, geom, prec)
    tune_set(N, geom, prec, alt, cur["grid_mult"])
    e = tune_get(N, geom, prec)["elems_per_group"]
    tune_set(N, geom, prec, cur["epb_alt"], cur["grid_mult"])
    return e


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, nargs="*", default=None)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args(argv)
    res = tune(orders=args.N or range(1, 16))
    if os.path.exists(args.out) and args.N:
        with open(args.out) as f:
            old = json.load(f)
        keep = [e for e in old.get("entries", []) if e["N"] not in set(args.N)]
        res["entries"] = sorted(keep + res["entries"], key=lambda e: (e["N"], e["geom"], e["prec"]))
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {args.out} ({len(res['entries'])} entries)")


if __name__ == "__main__":
    main()
