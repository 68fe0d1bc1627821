"""CPU checks of the C ABI: the library loads, exports every function the header declares, and
rejects invalid arguments with the documented status before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2504_07042_amd import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ax():
    import paper_2504_07042_amd as ax
    if not os.path.exists(ax.LIBPATH):
        pytest.fail("libaxhosfem.so not built (run __graft_entry__.build())")
    ax.lib()
    return ax


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            for m in re.finditer(r"^\s*(?:const\s+)?(?:int|char\s*\*|char|void)\s*\*?\s*(\w+)\s*\(", txt, re.M):
                names.add(m.group(1))
    return names


def test_exports_every_declared_symbol(ax):
    names = _declared()
    assert {"ax_local", "ax_local_precomputedG", "gs_assemble", "cg_solve"} <= names
    L = ctypes.CDLL(ax.LIBPATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_gll_matches_oracle(ax):
    for N in range(1, 16):
        xi, w, D = ax.gll(N)
        xo, wo, Do = oracle.gll(N)
        assert np.abs(xi - xo).max() <= 4e-16
        assert np.abs(w - wo).max() <= 4 * N * 1e-16
        assert np.abs(D - Do).max() <= 1e-13 * np.abs(Do).max()


def _call_local(ax, E=4, N=3, geom=0, nrhs=1, prec=0, X=1, Y=2, D=True, xi=True, w=True, geo=3):
    b = ax.Basis(3)
    L = ax.lib()
    return L.ax_local(E, N, geom, ctypes.c_void_p(geo) if geo else None,
                      ax._np_ptr(b.D) if D else None, ax._np_ptr(b.xi) if xi else None,
                      ax._np_ptr(b.w) if w else None, nrhs, prec,
                      ctypes.c_void_p(X) if X else None, ctypes.c_void_p(Y) if Y else None, None)


def test_ax_local_validation(ax):
    assert _call_local(ax, E=-1) == ax.AX_ERR_ARG
    assert _call_local(ax, nrhs=0) == ax.AX_ERR_ARG
    assert _call_local(ax, N=0) == ax.AX_ERR_UNSUPPORTED
    assert _call_local(ax, N=16) == ax.AX_ERR_UNSUPPORTED
    assert _call_local(ax, prec=7) == ax.AX_ERR_UNSUPPORTED
    assert _call_local(ax, geom=5) == ax.AX_ERR_UNSUPPORTED
    assert _call_local(ax, X=0) == ax.AX_ERR_ARG
    assert _call_local(ax, X=5, Y=5) == ax.AX_ERR_ARG
    assert _call_local(ax, D=False) == ax.AX_ERR_ARG
    assert _call_local(ax, xi=False) == ax.AX_ERR_ARG
    assert _call_local(ax, geo=0) == ax.AX_ERR_ARG
    assert _call_local(ax, E=0, X=0, Y=0, geo=0) == ax.AX_OK  # empty is a no-op
    assert _call_local(ax, E=-1) == ax.AX_ERR_ARG
    assert len(ax.lib().ax_last_error()) > 0


def test_precomputed_validation(ax):
    b = ax.Basis(2)
    L = ax.lib()
    assert L.ax_local_precomputedG(3, 2, None, ax._np_ptr(b.D), 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), None) == ax.AX_ERR_ARG
    assert L.ax_local_precomputedG(3, 2, ctypes.c_void_p(8), ax._np_ptr(b.D), 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == ax.AX_ERR_ARG
    assert L.ax_local_precomputedG(3, 99, ctypes.c_void_p(8), ax._np_ptr(b.D), 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), None) == ax.AX_ERR_UNSUPPORTED


def test_gs_validation_and_csr(ax):
    L = ax.lib()
    assert L.gs_assemble(4, 2, None, None, None, None, 9, 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), None) == ax.AX_ERR_UNSUPPORTED
    assert L.gs_assemble(4, 2, None, None, None, None, ax.GS_QT, 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), None) == ax.AX_ERR_ARG
    assert L.gs_assemble(4, 2, ctypes.c_void_p(3), None, None, None, ax.GS_Q, 1, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == ax.AX_ERR_ARG
    assert L.gs_assemble(-1, 2, None, None, None, None, ax.GS_Q, 1, 0, None, None, None) == ax.AX_ERR_ARG
    bad = np.array([0, 5], dtype=np.int32)
    with pytest.raises(ax.AxError):
        ax.gs_build_csr(bad, 3)
    l2g, ng, _ = meshgen.global_numbering(3, 2, 2, 3)
    gptr, gidx = ax.gs_build_csr(l2g, ng)
    assert gptr[0] == 0 and gptr[-1] == l2g.size
    for g in range(ng):
        loc = gidx[gptr[g]:gptr[g + 1]]
        assert np.array_equal(loc, np.nonzero(l2g == g)[0])


def test_tuning_roundtrip(ax):
    from paper_2504_07042_amd import autotune
    K, P = ax.AX_TUNE_TRILINEAR, ax.AX_FP64
    before = autotune.tune_get(7, K, P)
    try:
        autotune.tune_set(7, K, P, kernel=ax.AX_KERNEL_TILE, tile_alt=1, grid_mult=4)
        t = autotune.tune_get(7, K, P)
        assert (t["kernel_used"], t["elems_per_group"], t["block"], t["grid_mult"]) == (ax.AX_KERNEL_TILE, 2, 128, 4)
        autotune.tune_set(7, K, P, kernel=ax.AX_KERNEL_ITEM, item_alt=1, waves_alt=1)
        t = autotune.tune_get(7, K, P)
        assert (t["kernel_used"], t["elems_per_group"], t["block"], t["waves"]) == (ax.AX_KERNEL_ITEM, 2, 128, 3)
        autotune.tune_set(7, K, P, kernel=ax.AX_KERNEL_AUTO, item_alt=0, waves_alt=0)
        assert autotune.tune_get(7, K, P)["kernel_used"] == ax.AX_KERNEL_TILE      # N1 = 8: measured default
        assert autotune.tune_get(6, K, P)["kernel_used"] == ax.AX_KERNEL_ITEM
        # the partial form has a per-item kernel from N1 = 9 only
        autotune.tune_set(7, ax.AX_TUNE_PARTIAL, P, kernel=ax.AX_KERNEL_ITEM)
        assert autotune.tune_get(7, ax.AX_TUNE_PARTIAL, P)["kernel_used"] == ax.AX_KERNEL_TILE
        autotune.tune_set(7, ax.AX_TUNE_PARTIAL, P, kernel=ax.AX_KERNEL_AUTO)
        # batched: per-item, shape per order
        saved3 = autotune.tune_get(3, ax.AX_TUNE_BATCHED, ax.AX_FP32)
        autotune.tune_set(3, ax.AX_TUNE_BATCHED, ax.AX_FP32, kernel=ax.AX_KERNEL_AUTO, item_alt=1)
        t = autotune.tune_get(3, ax.AX_TUNE_BATCHED, ax.AX_FP32)
        assert (t["kernel_used"], t["elems_per_group"], t["block"], t["waves"]) == (ax.AX_KERNEL_ITEM, 8, 128, 5)
        autotune.tune_set(3, ax.AX_TUNE_BATCHED, ax.AX_FP32, **{k: saved3[k] for k in autotune.KNOBS})
        # the variants the tuner enumerates at N1 = 12: one tile shape (no alternative there) and
        # the per-item kernel in two shapes times two register budgets
        v = autotune._variants(11, K, ax.AX_FP32)
        assert len(v) == 5 and len({tuple(sorted(d.items())) for d in v}) == 5
        assert sum(d["kernel"] == ax.AX_KERNEL_ITEM for d in v) == 4
        assert len(autotune._variants(11, ax.AX_TUNE_STORED, ax.AX_FP32)) == 1
        # batched: two per-item shapes, the tile kernel over mesh slices, and over the work list
        # where the order has that form (FP64 up to N = 6)
        assert len(autotune._variants(3, ax.AX_TUNE_BATCHED, ax.AX_FP64)) == 4
        assert len(autotune._variants(7, ax.AX_TUNE_BATCHED, ax.AX_FP64)) == 3
        assert len(autotune._variants(7, ax.AX_TUNE_BATCHED, ax.AX_FP32)) == 4
        saved_b = {prec: autotune.tune_get(7, ax.AX_TUNE_BATCHED, prec) for prec in (ax.AX_FP64, ax.AX_FP32)}
        autotune.tune_set(7, ax.AX_TUNE_BATCHED, ax.AX_FP32, kernel=ax.AX_KERNEL_TILE, tile_alt=0)
        t = autotune.tune_get(7, ax.AX_TUNE_BATCHED, ax.AX_FP32)
        assert (t["kernel_used"], t["elems_per_group"], t["block"]) == (ax.AX_KERNEL_TILE, 1, 64)
        autotune.tune_set(7, ax.AX_TUNE_BATCHED, ax.AX_FP64, kernel=ax.AX_KERNEL_TILE, tile_alt=0)
        assert autotune.tune_get(7, ax.AX_TUNE_BATCHED, ax.AX_FP64)["kernel_used"] == ax.AX_KERNEL_ITEM
        autotune.tune_set(7, ax.AX_TUNE_BATCHED, ax.AX_FP64, kernel=ax.AX_KERNEL_TILE, tile_alt=1)
        t = autotune.tune_get(7, ax.AX_TUNE_BATCHED, ax.AX_FP64)
        assert (t["kernel_used"], t["elems_per_group"], t["block"]) == (ax.AX_KERNEL_TILE, 1, 64)
        for prec, sv in saved_b.items():
            autotune.tune_set(7, ax.AX_TUNE_BATCHED, prec, **{k: sv[k] for k in autotune.KNOBS})
    finally:
        autotune.tune_set(7, K, P, **{k: before[k] for k in autotune.KNOBS})
    assert autotune.tune_get(7, K, P) == before
    L = ax.lib()

    def raw(N, kind, prec, **kw):
        t = ax.AxTune(**dict(autotune.DEFAULT, **kw))
        return L.ax_tune_set(N, kind, prec, ctypes.byref(t))
    assert raw(7, K, P) == ax.AX_OK
    assert raw(7, K, P, kernel=3) == ax.AX_ERR_ARG
    assert raw(7, K, P, tile_alt=2) == ax.AX_ERR_ARG
    assert raw(7, K, P, waves_alt=-1) == ax.AX_ERR_ARG
    assert raw(7, K, P, grid_mult=0) == ax.AX_ERR_ARG
    assert raw(7, K, P, grid_mult=65) == ax.AX_ERR_ARG
    assert raw(16, K, P) == ax.AX_ERR_UNSUPPORTED
    assert raw(7, 6, P) == ax.AX_ERR_ARG
    assert raw(7, K, ax.AX_FP16_ACC32) == ax.AX_ERR_ARG
    assert raw(10, ax.AX_TUNE_BATCHED, P) == ax.AX_ERR_ARG
    assert L.ax_tune_set(7, K, P, None) == ax.AX_ERR_ARG
    assert L.ax_tune_get(7, K, P, None) == ax.AX_ERR_ARG


def test_cg_validation(ax):
    """cg_workspace_bytes validates the problem and options before any GPU work: a local node
    count beyond int32 local ids, a bad order and bad options are rejected."""
    L = ax.lib()
    b = ax.Basis(7)
    p = ax.AxProblem(E=32768, N=7, geom=ax.AX_TRILINEAR, geo=3, D=ax._np_ptr(b.D), xi=ax._np_ptr(b.xi),
                     w=ax._np_ptr(b.w), n_global=225 ** 3, l2g=5, gptr=6, gidx=7, mask=None)
    o = ax.AxCgOpts(rtol=1e-10, max_it=100, inner_prec=ax.AX_FP64, inner_rtol=0.1, max_outer=10,
                    workspace=None, workspace_bytes=0, use_graph=1, refine=ax.AX_REFINE_RELIABLE)
    n = ctypes.c_size_t(0)
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_OK
    assert n.value > 8 * 3 * 225 ** 3
    p.E = (2 ** 31) // 512 + 1          # 2^31 + 512 local nodes
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_ERR_UNSUPPORTED
    p.E, p.N = 64, 16
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_ERR_UNSUPPORTED
    p.N = 3
    o.rtol = 0.0
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_ERR_ARG
    o.rtol = 1e-10
    n0 = ctypes.c_size_t(0)
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n0)) == ax.AX_OK
    o.precond = ax.AX_PRECOND_JACOBI
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_OK
    assert n.value >= n0.value + 8 * p.n_global          # room for the inverse diagonal
    o.precond = 7
    assert L.cg_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), ctypes.byref(n)) == ax.AX_ERR_ARG


def test_partial_validation(ax):
    """ax_local_partial and ax_geom_lambda reject bad arguments before touching the GPU."""
    b = ax.Basis(3)
    L = ax.lib()
    D, xi, w = ax._np_ptr(b.D), ax._np_ptr(b.xi), ax._np_ptr(b.w)
    assert L.ax_local_partial(2, 3, None, None, D, xi, w, 1, ax.AX_FP64, 8, 16, None) == ax.AX_ERR_ARG
    assert L.ax_local_partial(2, 3, 8, 8, D, xi, w, 1, ax.AX_FP16_ACC32, 8, 16, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_local_partial(2, 3, 8, 8, D, None, w, 1, ax.AX_FP64, 8, 16, None) == ax.AX_ERR_ARG
    assert L.ax_local_partial(2, 16, 8, 8, D, xi, w, 1, ax.AX_FP64, 8, 16, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_local_partial(2, 3, 8, 8, D, xi, w, 1, ax.AX_FP64, 8, 8, None) == ax.AX_ERR_ARG
    assert L.ax_local_partial(0, 3, None, None, D, xi, w, 1, ax.AX_FP64, None, None, None) == ax.AX_OK
    assert L.ax_geom_lambda(2, 3, None, xi, w, ax.AX_FP64, 8, None) == ax.AX_ERR_ARG
    assert L.ax_geom_lambda(2, 3, 8, xi, w, ax.AX_FP16_ACC32, 8, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_geom_lambda(-1, 3, 8, xi, w, ax.AX_FP64, 8, None) == ax.AX_ERR_ARG


def test_helmholtz_validation(ax):
    b = ax.Basis(3)
    L = ax.lib()
    D, xi, w = ax._np_ptr(b.D), ax._np_ptr(b.xi), ax._np_ptr(b.w)
    assert L.ax_local_helmholtz(2, 3, 8, None, D, xi, w, 1, ax.AX_FP64, 8, 16, None) == ax.AX_ERR_ARG
    assert L.ax_local_helmholtz(2, 3, 8, 8, D, xi, w, 1, ax.AX_FP16_ACC32, 8, 16, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_local_helmholtz(2, 0, 8, 8, D, xi, w, 1, ax.AX_FP64, 8, 16, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_local_helmholtz(0, 3, None, None, D, xi, w, 1, ax.AX_FP64, None, None, None) == ax.AX_OK
    assert L.ax_helmholtz_factors(2, 3, 8, xi, w, None, 8, ax.AX_FP64, 8, None) == ax.AX_ERR_ARG
    assert L.ax_helmholtz_factors(2, 3, 8, xi, w, 8, 8, 7, 8, None) == ax.AX_ERR_UNSUPPORTED


def test_batched_noalloc_rejects_oversize_before_the_gpu(ax):
    """More meshes than the static work list holds, or a work list beyond its 8 MiB, is an
    argument error found on the host (nothing touches the device)."""
    b = ax.Basis(3)
    L = ax.lib()
    many = (ax.AxProblem * 5000)()
    for q in range(5000):
        many[q] = ax.AxProblem(0, 3, ax.AX_TRILINEAR, None, b.D.ctypes.data, b.xi.ctypes.data, b.w.ctypes.data,
                               0, None, None, None, None)
    xs = (ctypes.c_void_p * 5000)(*([8] * 5000))
    ys = (ctypes.c_void_p * 5000)(*([16] * 5000))
    assert L.ax_local_batched_noalloc(5000, many, 1, ax.AX_FP64, ctypes.cast(xs, ctypes.c_void_p),
                                      ctypes.cast(ys, ctypes.c_void_p), None, None) == ax.AX_ERR_ARG
    assert b"at most 4096" in L.ax_last_error()
    big = (ax.AxProblem * 1)(ax.AxProblem(1 << 30, 3, ax.AX_TRILINEAR, 64, b.D.ctypes.data, b.xi.ctypes.data,
                                          b.w.ctypes.data, 0, None, None, None, None))
    x1 = (ctypes.c_void_p * 1)(8)
    y1 = (ctypes.c_void_p * 1)(16)
    assert L.ax_local_batched_noalloc(1, big, 1, ax.AX_FP64, ctypes.cast(x1, ctypes.c_void_p),
                                      ctypes.cast(y1, ctypes.c_void_p), None, None) == ax.AX_ERR_ARG
    assert b"bytes of work list" in L.ax_last_error()


def test_probe_validation(ax):
    L = ax.lib()
    assert L.ax_probe_copy(None, ctypes.c_void_p(16), 64, None) == ax.AX_ERR_ARG
    assert L.ax_probe_copy(ctypes.c_void_p(16), ctypes.c_void_p(16), 64, None) == ax.AX_ERR_ARG
    assert L.ax_probe_copy(ctypes.c_void_p(16), ctypes.c_void_p(64), 40, None) == ax.AX_ERR_ARG
    assert L.ax_probe_copy(ctypes.c_void_p(8), ctypes.c_void_p(64), 64, None) == ax.AX_ERR_ARG
    assert L.ax_probe_copy(None, None, 0, None) == ax.AX_OK
    fl = ctypes.c_double()
    assert L.ax_probe_compute(0, 0, ctypes.c_void_p(16), ctypes.byref(fl), None) == ax.AX_ERR_ARG
    assert L.ax_probe_compute(0, 10, None, ctypes.byref(fl), None) == ax.AX_ERR_ARG
    assert L.ax_probe_compute(0, 10, ctypes.c_void_p(16), None, None) == ax.AX_ERR_ARG


def test_batched_launch_rejects_foreign_plan(ax):
    """A plan whose shape variants were not written by ax_batched_prepare is refused on the host."""
    L = ax.lib()
    plan = ax.AxBatchPlan()
    plan.prec = ax.AX_FP64
    plan.n_items = 5
    plan.order_variant[4] = 7
    assert L.ax_local_batched(ctypes.byref(plan), ctypes.c_void_p(256), None) == ax.AX_ERR_ARG
    assert b"shape variant" in L.ax_last_error()


def test_check_mesh_validation(ax):
    L = ax.lib()
    b = ax.Basis(3)
    bad = ctypes.c_int64(5)
    dmin = ctypes.c_double(0.0)
    xi = ax._np_ptr(b.xi)
    assert L.ax_check_mesh(-1, 3, ctypes.c_void_p(8), xi, None, None, None) == ax.AX_ERR_ARG
    assert L.ax_check_mesh(4, 0, ctypes.c_void_p(8), xi, None, None, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_check_mesh(4, 16, ctypes.c_void_p(8), xi, None, None, None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_check_mesh(4, 3, ctypes.c_void_p(8), None, None, None, None) == ax.AX_ERR_ARG
    assert L.ax_check_mesh(4, 3, None, xi, ctypes.byref(bad), ctypes.byref(dmin), None) == ax.AX_ERR_ARG
    assert bad.value == -1 and dmin.value == float("inf")
    # an empty mesh is valid and touches no device
    bad.value = 5
    assert L.ax_check_mesh(0, 3, None, xi, ctypes.byref(bad), ctypes.byref(dmin), None) == ax.AX_OK
    assert bad.value == -1 and dmin.value == float("inf")


def test_tuning_cache_load_is_tolerant(ax, tmp_path):
    """The cache loader applies valid entries, skips entries of another format or an unknown kind,
    and reports whether the cache was measured on the present kernel sources."""
    import json
    from paper_2504_07042_amd import autotune
    K, P = ax.AX_TUNE_TRILINEAR, ax.AX_FP64
    before = autotune.tune_get(5, K, P)
    path = tmp_path / "cache.json"
    entries = [
        {"N": 5, "kind": "trilinear", "prec": "fp64", "kernel": ax.AX_KERNEL_TILE, "tile_alt": 1, "item_alt": 0,
         "waves_alt": 0, "grid_mult": 4},
        {"N": 5, "geom": "trilinear", "prec": "fp64", "epb_alt": 1, "grid_mult": 4},       # older format
        {"N": 5, "kind": "nonsense", "prec": "fp64", "kernel": 0, "grid_mult": 1},
        {"N": 5, "kind": "stored", "prec": "fp64", "kernel": 0, "tile_alt": 0, "item_alt": 0,
         "waves_alt": 0, "grid_mult": 99},                                                   # invalid value
    ]
    path.write_text(json.dumps({"arch": "gfx950", "sources_sha256": "0" * 64, "entries": entries}))
    try:
        assert autotune.load(str(path)) == 1
        t = autotune.tune_get(5, K, P)
        assert (t["kernel_used"], t["tile_alt"], t["grid_mult"]) == (ax.AX_KERNEL_TILE, 1, 4)
        assert autotune.cache_status(str(path)) == "stale"
        assert autotune.cache_status(str(tmp_path / "absent.json")) == "absent"
    finally:
        autotune.tune_set(5, K, P, **{k: before[k] for k in autotune.KNOBS})
    assert autotune.tune_get(5, K, P) == before


def test_gathered_energy_validation(ax):
    """The energy variant of the gathering operator rejects its own missing buffers (and the
    gathering operator's bad arguments) before any launch."""
    L = ax.lib()
    b = ax.Basis(3)
    D, xi, w = ax._np_ptr(b.D), ax._np_ptr(b.xi), ax._np_ptr(b.w)
    v = ctypes.c_void_p

    def call(E=4, work=56, energy=64, l2g=8, ng=10, Xg=16, Y=24, N=3):
        return L.ax_local_gathered_energy(E, N, ax.AX_TRILINEAR, v(32), D, xi, w, v(l2g) if l2g else None, ng,
                                          v(Xg) if Xg else None, v(Y) if Y else None, v(work) if work else None,
                                          v(energy) if energy else None, None)

    assert call(energy=0) == ax.AX_ERR_ARG
    assert call(work=0) == ax.AX_ERR_ARG
    assert call(l2g=0) == ax.AX_ERR_ARG
    assert call(ng=0) == ax.AX_ERR_ARG
    assert call(Xg=16, Y=16) == ax.AX_ERR_ARG
    assert call(N=0) == ax.AX_ERR_UNSUPPORTED
    assert len(L.ax_last_error()) > 0


def test_recorded_measurements_match_the_sources():
    """The shipped launch-variant cache and the headline kernel's recorded HBM traffic were both
    measured on the kernel sources as they are: a change to those sources must be followed by a
    re-run of the tuner and of the FETCH_SIZE / WRITE_SIZE passes (the bench line would otherwise
    report a stale cache and a null traffic figure)."""
    import sys
    from paper_2504_07042_amd import autotune
    assert autotune.cache_status() == "current"
    sys.path.insert(0, ROOT)
    import bench
    traffic = bench.measured_traffic(7, 32768)
    assert traffic is not None
    # calibrated bytes per launch within 2 % of the algorithmic 32768 x 8384 B
    assert abs(traffic / (32768 * 8384) - 1.0) < 0.02
