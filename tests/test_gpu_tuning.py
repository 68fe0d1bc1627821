"""Every launch variant the tuning table can select computes the operator: each variant of each
kernel (tile or per-item; work-group shape; register budget; persistent grid) is checked against
the oracle, and variants of one kernel against each other bit for bit (they differ only in how
elements are grouped and scheduled, not in the arithmetic per element).  The batched kernels'
two per-item work-group shapes likewise, and their tile kernel (over the work list and over mesh
slices) against the single-mesh tile kernel."""
import numpy as np
import pytest

import oracle
from gpu_util import check_bound, check_fp64, cond_j_per_element, fp32_bound, report
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kind", ["trilinear", "partial"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [1, 2, 4, 5, 7, 8, 9, 10, 11, 12, 14, 15])
def test_every_variant(ax, N, prec, kind):
    import torch
    from paper_2504_07042_amd import autotune
    P = ax.AX_FP64 if prec == "fp64" else ax.AX_FP32
    K = autotune.KINDS[kind]
    m = meshgen.jittered_hex(5, 4, 3, alpha=0.15, seed=300 + N)     # 60 elements: ragged groups
    b = ax.Basis(N)
    X = meshgen.random_nodal(m.E, N, nrhs=2, seed=N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Yref, env = oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X)
    V = _dev(m.verts)
    Xd = _dev(X) if P == ax.AX_FP64 else _dev(X).float()
    lam = ax.geom_lambda(V, b, P) if kind == "partial" else None
    if P == ax.AX_FP32:
        factor = fp32_bound(N, cond_j_per_element(m.verts, N))[None, :, None]
    saved = autotune.tune_get(N, K, P)
    by_kernel = {}
    try:
        variants = autotune._variants(N, K, P)
        assert variants
        for v in variants:
            for gm in (1, 3):
                autotune.tune_set(N, K, P, grid_mult=gm, **v)
                info = autotune.tune_get(N, K, P)
                if kind == "partial":
                    Y = ax.ax_local_partial(Xd, V, lam, b, P)
                else:
                    Y = ax.ax_local(Xd, V, b, ax.AX_TRILINEAR, P)
                torch.cuda.synchronize()
                Yh = Y.double().cpu().numpy()
                tag = (f"tuning N={N} {prec} {kind} kernel={info['kernel_used']} epg={info['elems_per_group']} "
                       f"block={info['block']} waves={info['waves']} grid={gm}")
                if P == ax.AX_FP64:
                    check_fp64(Yh, Yref, env, tag=tag)
                else:
                    check_bound(Yh, Yref, env, factor, tag=tag)
                by_kernel.setdefault(info["kernel_used"], []).append((tag, Yh))
    finally:
        autotune.tune_set(N, K, P, **{k: saved[k] for k in autotune.KNOBS})
    for runs in by_kernel.values():
        for tag, Yh in runs[1:]:
            assert np.array_equal(Yh, runs[0][1]), f"{tag} differs bitwise from {runs[0][0]}"
    report("tuning_variants", N=N, prec=prec, kind=kind, kernels=sorted(by_kernel),
           runs=sum(len(r) for r in by_kernel.values()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_shapes(ax, prec):
    import torch
    from paper_2504_07042_amd import autotune
    P = ax.AX_FP64 if prec == "fp64" else ax.AX_FP32
    specs = [(1, (5, 4, 4)), (2, (4, 4, 3)), (3, (3, 4, 5)), (4, (4, 3, 3)), (5, (3, 3, 4)), (6, (4, 3, 2)),
             (7, (3, 3, 3)), (8, (3, 2, 3)), (9, (2, 3, 3)), (7, (2, 2, 1))]
    meshes, X, Yref, env, fac = [], [], [], [], []
    for q, (N, dims) in enumerate(specs):
        m = meshgen.jittered_hex(*dims, alpha=0.12, seed=90 + q)
        b = ax.Basis(N)
        meshes.append((_dev(m.verts), b))
        x = meshgen.random_nodal(m.E, N, nrhs=2, seed=q)
        X.append(_dev(x) if P == ax.AX_FP64 else _dev(x).float())
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        Yref.append(oracle.ax_local(D, G, x))
        env.append(oracle.ax_envelope(D, G, x))
        if P == ax.AX_FP32:
            fac.append(fp32_bound(N, cond_j_per_element(m.verts, N))[None, :, None])
    saved = {N: autotune.tune_get(N, ax.AX_TUNE_BATCHED, P) for N in range(1, 10)}
    saved_tri = {N: autotune.tune_get(N, ax.AX_TUNE_TRILINEAR, P) for N in range(1, 10)}
    outs = {}
    try:
        # shape variants 0 and 1 of the per-item kernel, 2 the tile kernel over the work list, 3 the
        # tile kernel over mesh slices
        for alt in (0, 1, 2, 3):
            for N in range(1, 10):
                if alt == 2:
                    autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, kernel=ax.AX_KERNEL_TILE, tile_alt=0, item_alt=0,
                                      grid_mult=1)
                elif alt == 3:
                    autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, kernel=ax.AX_KERNEL_TILE, tile_alt=1, grid_mult=1)
                else:
                    autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, kernel=ax.AX_KERNEL_AUTO, item_alt=alt)
            Y = [torch.empty_like(x) for x in X]
            plan = ax.BatchedAxLocal(meshes, X, Y, P)
            # the tile kernel exists up to N = 6 in FP64 and N = 9 in FP32 (per-item shape 0 beyond)
            top = 6 if P == ax.AX_FP64 else 9
            want = [2 if N <= top else 0 for N in range(1, 10)] if alt == 2 else [alt] * 9
            assert list(plan.plan.order_variant)[2:11] == want
            plan.launch()
            torch.cuda.synchronize()
            outs[alt] = [y.double().cpu().numpy() for y in Y]
            for q, (N, _) in enumerate(specs):
                tag = f"batched shape={alt} {prec} mesh={q} N={N}"
                if P == ax.AX_FP64:
                    check_fp64(outs[alt][q], Yref[q], env[q], tag=tag)
                else:
                    check_bound(outs[alt][q], Yref[q], env[q], fac[q], tag=tag)
        # the tile kernel over the work list computes each element exactly as the single-mesh
        # tile kernel does
        for N in range(1, 10):
            autotune.tune_set(N, ax.AX_TUNE_TRILINEAR, P, kernel=ax.AX_KERNEL_TILE, tile_alt=0)
        for q, (N, _) in enumerate(specs):
            Ys = ax.ax_local(X[q], meshes[q][0], meshes[q][1], ax.AX_TRILINEAR, P).double().cpu().numpy()
            assert np.array_equal(outs[3][q], Ys), q
            if N <= top:
                assert np.array_equal(outs[2][q], Ys), q
    finally:
        for N, s in saved.items():
            autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, **{k: s[k] for k in autotune.KNOBS})
        for N, s in saved_tri.items():
            autotune.tune_set(N, ax.AX_TUNE_TRILINEAR, P, **{k: s[k] for k in autotune.KNOBS})
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
