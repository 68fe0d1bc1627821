"""The allocation-free batched launch (ax_local_batched_noalloc) against the workspace path
(ax_batched_prepare + ax_local_batched) through the C ABI: two calls in a row on the same device
array, the second with a smaller batch, each equal bit for bit to the workspace path (same
kernels, same inputs), in FP64 and FP32."""
import numpy as np
import pytest

from paper_2504_07042_amd import meshgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_07042_amd as ax
    ax.lib()
    return ax


def _batch(ax, specs, nrhs, dtype, seed):
    import torch
    meshes, X = [], []
    for q, (N, grid) in enumerate(specs):
        m = meshgen.jittered_hex(*grid, alpha=0.1, seed=seed + q)
        meshes.append((torch.from_numpy(m.verts).cuda(), ax.Basis(N)))
        X.append(meshgen.random_nodal_device(m.E, N, nrhs, seed=seed + q, device="cuda", dtype=dtype))
    return meshes, X


@pytest.mark.parametrize("form", ["tuned", "slices"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_path(ax, prec, form):
    """`form`: the launch variants of the tuning table, or every order forced to the tile kernel
    over mesh slices (each mesh's work-group count then comes from the same split in both
    paths)."""
    from paper_2504_07042_amd import autotune
    p = ax.AX_FP64 if prec == "fp64" else ax.AX_FP32
    saved = {N: autotune.tune_get(N, ax.AX_TUNE_BATCHED, p) for N in (3, 5, 7, 9)}
    if form == "slices":
        for N in saved:
            autotune.tune_set(N, ax.AX_TUNE_BATCHED, p, kernel=ax.AX_KERNEL_TILE, tile_alt=1)
    try:
        _noalloc_vs_workspace(ax, prec, p)
    finally:
        for N, sv in saved.items():
            autotune.tune_set(N, ax.AX_TUNE_BATCHED, p, **{k: sv[k] for k in autotune.KNOBS})


def _noalloc_vs_workspace(ax, prec, p):
    import torch
    dtype = torch.float64 if prec == "fp64" else torch.float32
    big = [(3, (9, 8, 7)), (5, (6, 5, 5)), (7, (5, 4, 4)), (9, (3, 4, 3)), (3, (2, 2, 1)), (7, (7, 6, 5))]
    small = [(5, (2, 3, 2)), (3, (1, 1, 3))]
    for call, specs in enumerate((big, small)):
        print(f"[no-alloc] {prec} call {call}: {len(specs)} meshes {specs}", flush=True)
        meshes, X = _batch(ax, specs, 3, dtype, seed=10 * call + 1)
        Yw = [torch.full_like(x, float("nan")) for x in X]
        Yn = [torch.full_like(x, float("nan")) for x in X]
        ax.BatchedAxLocal(meshes, X, Yw, p).launch()
        ax.batched_noalloc(meshes, X, Yn, p)
        torch.cuda.synchronize()
        for q in range(len(specs)):
            assert torch.isfinite(Yn[q]).all()
            assert torch.equal(Yn[q], Yw[q]), (call, q)
