"""Autotuner for the AxLocal launch variants on gfx950.

For each (order N, tuning kind, precision) it times every launch variant the library can select
at run time (``ax_tune_set``):

* the kernel: the prefetching tile kernel or the per-item kernel (where the form has one);
* the tile kernel's elements per work-group (default or alternative shape);
* the per-item kernels' work-group shape (256 lanes or the order's alternative) and, for the
  single-mesh per-item kernel, its register budget (default or alternative waves per SIMD);
* the persistent grid (1, 2, 4 or 8 times the resident work-group capacity);

on a synthetic mesh of about 2^24 local nodes (four rotating X/Y pairs, as the benchmark times
them, so that the vectors do not stay in the 256 MB Infinity Cache), keeps the fastest when it
beats the default by more than the noise margin, and writes a JSON cache stamped with the
SHA-256 of the kernel sources it was measured on.  ``load()`` pushes a cache into the library; the package calls it on import.  Every
variant gives the same result up to rounding (bitwise the same for one kernel).

    python -m paper_2504_07042_amd.autotune            # tune everything, write the cache
    python -m paper_2504_07042_amd.autotune --N 7      # some orders only (merged into the cache)
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import itertools
import json
import os
import time

from . import (AX_FP32, AX_FP64, AX_KERNEL_AUTO, AX_KERNEL_ITEM, AX_KERNEL_TILE, AX_PARALLELEPIPED,
               AX_TRILINEAR, AX_TUNE_BATCHED, AX_TUNE_HELMHOLTZ, AX_TUNE_PARALLELEPIPED, AX_TUNE_PARTIAL,
               AX_TUNE_STORED, AX_TUNE_TRILINEAR, AxTune, Basis, _check, lib)

PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(PKG, "tuning_gfx950.json")
KINDS = {"trilinear": AX_TUNE_TRILINEAR, "parallelepiped": AX_TUNE_PARALLELEPIPED, "stored": AX_TUNE_STORED,
         "partial": AX_TUNE_PARTIAL, "helmholtz": AX_TUNE_HELMHOLTZ, "batched": AX_TUNE_BATCHED}
PRECS = {"fp64": AX_FP64, "fp32": AX_FP32}
KNOBS = ("kernel", "tile_alt", "item_alt", "waves_alt", "grid_mult")
DEFAULT = {"kernel": AX_KERNEL_AUTO, "tile_alt": 0, "item_alt": 0, "waves_alt": 0, "grid_mult": 2}
GRID_MULTS = (1, 2, 4, 8)
MARGIN = 0.01      # a variant replaces the default only if it is this much faster


# The sources the tuned launches depend on: the AxLocal kernels (tile, per-item, batched), their
# shared headers, the dispatch and the tuning table.  The solver, gather-scatter, set-up and probe
# sources do not change what the tuner times.
TUNED_SOURCES = ("ax_internal.h", "ax_kernels.h", "geom.h", "ax_local_impl.h", "ax_local_f64.hip",
                 "ax_local_f32.hip", "item.h", "item_f64.hip", "item_f32.hip", "batched.hip", "ax_local.hip",
                 "ax_common.cpp")


def source_hash() -> str:
    """SHA-256 over the sources the tuned launches depend on (TUNED_SOURCES)."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    for f in TUNED_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def tune_get(N: int, kind: int, prec: int) -> dict:
    t = AxTune()
    _check(lib().ax_tune_get(N, kind, prec, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in AxTune._fields_}


def tune_set(N: int, kind: int, prec: int, **knobs):
    """Set some knobs of one entry (the others keep their current values)."""
    cur = tune_get(N, kind, prec)
    cur.update(knobs)
    t = AxTune(**{k: int(cur[k]) for k in KNOBS})
    _check(lib().ax_tune_set(N, kind, prec, ctypes.byref(t)))


def cache_status(path: str = CACHE) -> str:
    """'current' (stamped with the present sources), 'stale' or 'absent'."""
    if not os.path.exists(path):
        return "absent"
    with open(path) as f:
        data = json.load(f)
    return "current" if data.get("sources_sha256") == source_hash() else "stale"


def load(path: str = CACHE) -> int:
    """Apply a tuning cache; returns the number of entries applied (0 if there is none).  A stale
    cache is applied too: every variant it names is valid, only possibly no longer the fastest."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for ent in data.get("entries", []):
        if ent.get("kind") not in KINDS or ent.get("prec") not in PRECS:
            continue
        try:
            tune_set(ent["N"], KINDS[ent["kind"]], PRECS[ent["prec"]], **{k: ent[k] for k in KNOBS if k in ent})
            n += 1
        except Exception:   # an entry of an older format: keep the default
            pass
    return n


def _variants(N: int, kind: int, prec: int):
    """Every distinct launch variant of one entry (as knob dicts, without the grid)."""
    saved = tune_get(N, kind, prec)
    out, seen = [], set()
    try:
        for kern, ta, ia, wa in itertools.product((AX_KERNEL_TILE, AX_KERNEL_ITEM), (0, 1), (0, 1), (0, 1)):
            tune_set(N, kind, prec, kernel=kern, tile_alt=ta, item_alt=ia, waves_alt=wa)
            r = tune_get(N, kind, prec)
            if r["kernel_used"] != kern:
                continue
            key = (r["kernel_used"], r["elems_per_group"], r["block"], r["waves"],
                   # batched: the tile kernel walks the work list (tile_alt 0) or mesh slices (1)
                   ta if kind == AX_TUNE_BATCHED and kern == AX_KERNEL_TILE else 0)
            if key in seen:
                continue
            seen.add(key)
            out.append({"kernel": kern, "tile_alt": ta, "item_alt": ia, "waves_alt": wa})
    finally:
        tune_set(N, kind, prec, **{k: saved[k] for k in KNOBS})
    return out


def _time_configs(fns, cands, apply, rounds=3, reps=12, warmup=4):
    """Interleaved timing: each round times every config; the best round per config counts."""
    import torch
    best = [float("inf")] * len(cands)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(rounds):
        for q, cfg in enumerate(cands):
            apply(cfg)
            for w in range(warmup):
                fns[w % len(fns)]()
            ev[0].record()
            for r in range(reps):
                fns[r % len(fns)]()
            ev[1].record()
            ev[1].synchronize()
            best[q] = min(best[q], ev[0].elapsed_time(ev[1]) * 1e-3 / reps)
    return best


NBUF = 4          # rotating X/Y pairs
BATCH_COLS = 8    # columns of the batched workload


def _workloads(N, prec, target_nodes, kinds):
    """Launch closures per tuning kind on NBUF rotating X/Y pairs of about target_nodes nodes."""
    import torch

    from . import (BatchedAxLocal, ax_local, ax_local_helmholtz, ax_local_partial, ax_local_precomputedG,
                   geom_factors, geom_lambda, helmholtz_factors, meshgen, parallelepiped_factors)
    b = Basis(N)
    NP = (N + 1) ** 3
    grid = meshgen.grid_for_nodes(N, target_nodes)
    m = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
    V = torch.from_numpy(m.verts).cuda()
    dt = torch.float64 if prec == AX_FP64 else torch.float32
    Xs = [meshgen.random_nodal_device(m.E, N, seed=N + q, dtype=dt) for q in range(NBUF)]
    Ys = [torch.empty_like(x) for x in Xs]
    work = {}
    if "trilinear" in kinds:
        work["trilinear"] = [lambda q=q: ax_local(Xs[q], V, b, AX_TRILINEAR, prec, out=Ys[q]) for q in range(NBUF)]
    if "parallelepiped" in kinds:
        pm, _ = meshgen.parallelepiped_hex(*grid, seed=2)
        h = parallelepiped_factors(torch.from_numpy(pm.verts).cuda())
        work["parallelepiped"] = [lambda q=q: ax_local(Xs[q], h, b, AX_PARALLELEPIPED, prec, out=Ys[q])
                                  for q in range(NBUF)]
    if "stored" in kinds:
        G, _ = geom_factors(V, b, prec)
        work["stored"] = [lambda q=q: ax_local_precomputedG(Xs[q], G, b, prec, out=Ys[q]) for q in range(NBUF)]
    if "partial" in kinds:
        lam = geom_lambda(V, b, prec)
        work["partial"] = [lambda q=q: ax_local_partial(Xs[q], V, lam, b, prec, out=Ys[q]) for q in range(NBUF)]
    if "helmholtz" in kinds:
        l0 = torch.ones((m.E, NP), dtype=torch.float64, device="cuda")
        l1 = torch.full((m.E, NP), 0.5, dtype=torch.float64, device="cuda")
        L23 = helmholtz_factors(V, l0, l1, b, prec)
        del l0, l1
        work["helmholtz"] = [lambda q=q: ax_local_helmholtz(Xs[q], V, L23, b, prec, out=Ys[q]) for q in range(NBUF)]
    if "batched" in kinds and N <= 9:
        # eight meshes of this order of uneven size (the batched kernels' work lists) with
        # BATCH_COLS columns, as the batched benchmark runs them
        sizes = [max(1, m.E * f // 36) for f in (8, 7, 6, 5, 4, 3, 2, 1)]
        meshes, off = [], 0
        for s in sizes:
            meshes.append((V[off:off + s], b))
            off += s
        Xb = [meshgen.random_nodal_device(m.E, N, BATCH_COLS, seed=N + q, dtype=dt) for q in range(NBUF)]
        Yb = [torch.empty_like(x) for x in Xb]
        views = [[x[:, a:a + s] for a, s in zip(itertools.accumulate([0] + sizes[:-1]), sizes)] for x in Xb]
        outs = [[y[:, a:a + s] for a, s in zip(itertools.accumulate([0] + sizes[:-1]), sizes)] for y in Yb]
        work["batched"] = (meshes, views, outs, BATCH_COLS)
    return m.E * NP, work


def tune(orders=range(1, 16), kinds=tuple(KINDS), precs=tuple(PRECS), target_nodes=1 << 24, verbose=True):
    import torch

    from . import BatchedAxLocal
    entries = []
    for N in orders:
        for pname in precs:
            prec = PRECS[pname]
            ndof, work = _workloads(N, prec, target_nodes, kinds)
            for kname in kinds:
                if kname not in work:
                    continue
                kind = KINDS[kname]
                variants = _variants(N, kind, prec)
                cands = [dict(v, grid_mult=g) for v in variants for g in GRID_MULTS]
                cands.insert(0, dict(DEFAULT))
                if kname == "batched":
                    meshes, views, outs, ncol = work["batched"]
                    plans = {}

                    def fn_for(cfg):
                        # a plan keeps the kernel and shape it was prepared with: one per variant
                        key = (cfg["kernel"], cfg["item_alt"], cfg["tile_alt"])
                        if key not in plans:
                            tune_set(N, kind, prec, kernel=cfg["kernel"], item_alt=cfg["item_alt"],
                                     tile_alt=cfg["tile_alt"])
                            plans[key] = [BatchedAxLocal(meshes, list(views[q]), list(outs[q]), prec)
                                          for q in range(NBUF)]
                        return [p.launch for p in plans[key]]
                    times = []
                    for cfg in cands:
                        fns = fn_for(cfg)
                        times.append(_time_configs(fns, [cfg], lambda c: tune_set(N, kind, prec, **c))[0])
                    del plans
                else:
                    times = _time_configs(work[kname], cands, lambda c: tune_set(N, kind, prec, **c))
                t_def = times[0]
                if kname == "batched":
                    times = [t / ncol for t in times]   # per column, as ndof counts one
                    t_def = times[0]
                q = min(range(len(cands)), key=lambda i: times[i])
                chosen = cands[q] if times[q] < (1.0 - MARGIN) * t_def else cands[0]
                t_best = times[q] if chosen is cands[q] else t_def
                tune_set(N, kind, prec, **chosen)
                info = tune_get(N, kind, prec)
                ent = {"N": N, "kind": kname, "prec": pname, **{k: info[k] for k in KNOBS},
                       "kernel_used": info["kernel_used"], "elems_per_group": info["elems_per_group"],
                       "block": info["block"], "waves": info["waves"], "variants_timed": len(cands),
                       "GDOFs": round(ndof / t_best / 1e9, 2), "GDOFs_default": round(ndof / t_def / 1e9, 2)}
                entries.append(ent)
                if verbose:
                    print(json.dumps(ent), flush=True)
            del work
            torch.cuda.empty_cache()
    return {"arch": "gfx950", "sources_sha256": source_hash(), "target_nodes": target_nodes,
            "created": time.strftime("%Y-%m-%d"), "margin": MARGIN, "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, nargs="*", default=None)
    ap.add_argument("--kinds", nargs="*", default=list(KINDS), choices=list(KINDS))
    ap.add_argument("--prec", nargs="*", default=list(PRECS), choices=list(PRECS))
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args(argv)
    res = tune(orders=args.N or range(1, 16), kinds=tuple(args.kinds), precs=tuple(args.prec))
    if os.path.exists(args.out) and (args.N or len(args.kinds) < len(KINDS) or len(args.prec) < len(PRECS)):
        with open(args.out) as f:
            old = json.load(f)
        new_keys = {(e["N"], e["kind"], e["prec"]) for e in res["entries"]}
        keep = [e for e in old.get("entries", []) if "kind" in e and (e["N"], e["kind"], e["prec"]) not in new_keys]
        res["entries"] = sorted(keep + res["entries"], key=lambda e: (e["N"], e["kind"], e["prec"]))
        if old.get("sources_sha256") != res["sources_sha256"] and keep:
            res["sources_sha256_note"] = "entries not re-timed in this run were measured on other sources"
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {args.out} ({len(res['entries'])} entries)")


if __name__ == "__main__":
    main()
