"""GPU CG and mixed-precision iterative refinement against the oracle: the oracle solves the
same system in FP64 and recomputes the true residual of every GPU solution."""
import numpy as np
import pytest

import oracle
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


def _problem(ax, N, grid, alpha=0.1, seed=4):
    import torch
    m = meshgen.jittered_hex(*grid, alpha=alpha, seed=seed)
    l2g, ng, mask = meshgen.global_numbering(*grid, N)
    b = ax.Basis(N)
    gs = ax.GatherScatter(l2g, ng, mask)
    V = torch.from_numpy(m.verts).cuda()
    prob = ax.Problem(V, b, gs)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    rhs, u = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
    return m, prob, (D, G, l2g, ng, mask), rhs


def _oracle_rel_res(N, ref, rhs, x):
    D, G, l2g, ng, mask = ref
    r = rhs - oracle.apply_A(N, D, G, l2g, ng, mask, x)
    return np.linalg.norm(r) / np.linalg.norm(rhs)


def test_apply_matches_oracle(ax):
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (3, 2, 2))
    D, G, l2g, ng, mask = ref
    x = np.random.default_rng(1).uniform(-1, 1, ng)
    y = prob.apply(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    yo = oracle.apply_A(N, D, G, l2g, ng, mask, x)
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)


@pytest.mark.parametrize("N,grid", [(3, (3, 3, 3)), (5, (2, 3, 2))])
def test_cg_fp64_matches_oracle(ax, N, grid):
    import torch
    m, prob, ref, rhs = _problem(ax, N, grid)
    xg, rep = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-10)
    assert rep["status"] == "AX_OK", rep
    x = xg.cpu().numpy()[0]
    assert _oracle_rel_res(N, ref, rhs, x) <= 1e-10
    D, G, l2g, ng, mask = ref
    xo, it, rel = oracle.cg(N, D, G, l2g, ng, mask, rhs, rtol=1e-10)
    assert np.abs(x - xo).max() <= 1e-8 * np.abs(xo).max()
    # same algorithm and scalars: iteration counts agree up to rounding drift
    assert abs(rep["iterations"] - it) <= max(2, it // 100), (rep["iterations"], it)


@pytest.mark.parametrize("inner", ["fp32", "fp16"])
def test_mixed_refinement_reaches_fp64_residual(ax, inner):
    import torch
    N = 4 if inner == "fp32" else 7
    m, prob, ref, rhs = _problem(ax, N, (3, 3, 3) if inner == "fp32" else (2, 2, 2))
    ip = {"fp32": ax.AX_FP32, "fp16": ax.AX_FP16_ACC32}[inner]
    xg, rep = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-10, inner_prec=ip,
                          inner_rtol=1e-5 if inner == "fp32" else 1e-2)
    assert rep["status"] == "AX_OK", rep
    assert rep["outer_it"] >= 2
    assert _oracle_rel_res(N, ref, rhs, xg.cpu().numpy()[0]) <= 1e-10


@pytest.mark.parametrize("inner", ["fp32", "fp16"])
def test_reliable_updates_reach_fp64_residual(ax, inner):
    """Mixed precision with reliable updates: one reduced-precision recurrence, FP64 residual
    replacements; the FP64 true residual reaches the target in about as many iterations as plain
    FP64 CG (FP32) and the oracle confirms the residual of the solution."""
    import torch
    N = 4 if inner == "fp32" else 7
    m, prob, ref, rhs = _problem(ax, N, (3, 3, 3) if inner == "fp32" else (2, 2, 2))
    ip = {"fp32": ax.AX_FP32, "fp16": ax.AX_FP16_ACC32}[inner]
    bd = torch.from_numpy(rhs[None]).cuda()
    _, r64 = ax.cg_solve(prob, bd, rtol=1e-10)
    xg, rep = ax.cg_solve(prob, bd, rtol=1e-10, inner_prec=ip, inner_rtol=0.1, refine=ax.AX_REFINE_RELIABLE)
    assert rep["status"] == "AX_OK", rep
    assert rep["outer_it"] >= 2
    assert _oracle_rel_res(N, ref, rhs, xg.cpu().numpy()[0]) <= 1e-10
    if inner == "fp32":
        assert rep["iterations"] <= 1.25 * r64["iterations"] + 8, (rep, r64)


def test_multi_rhs_and_warm_start(ax):
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (2, 2, 3))
    D, G, l2g, ng, mask = ref
    b2 = np.stack([rhs, 0.5 * rhs + np.where(mask == 1, 0.0, 1.0)])
    bd = torch.from_numpy(b2).cuda()
    xg, rep = ax.cg_solve(prob, bd, rtol=1e-10)
    assert rep["status"] == "AX_OK"
    for c in range(2):
        assert _oracle_rel_res(N, ref, b2[c], xg.cpu().numpy()[c]) <= 1e-10
    # resume from the solution: nothing left to do
    x2, rep2 = ax.cg_solve(prob, bd, x=xg.clone(), rtol=1e-10)
    assert rep2["status"] == "AX_OK" and rep2["iterations"] == 0


def test_not_converged_and_breakdown(ax):
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (2, 2, 2))
    _, rep = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-12, max_it=3)
    assert rep["status"] == "AX_ERR_NOT_CONVERGED"
    bad = rhs.copy()
    bad[np.nonzero(ref[4] == 0)[0][0]] = np.nan
    _, rep = ax.cg_solve(prob, torch.from_numpy(bad[None]).cuda(), rtol=1e-10)
    assert rep["status"] == "AX_ERR_BREAKDOWN"


def test_masked_rhs_rejected(ax):
    """A right-hand side that is nonzero on a Dirichlet node cannot be matched by the assembled
    operator (its row there is zero): the solver rejects it before iterating."""
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (2, 2, 2))
    bad = rhs.copy()
    bad[np.nonzero(ref[4] == 1)[0][0]] = 1.0
    with pytest.raises(ax.AxError) as ei:
        ax.cg_solve(prob, torch.from_numpy(bad[None]).cuda(), rtol=1e-10)
    assert ei.value.code == ax.AX_ERR_ARG


def test_graph_replay_equals_eager(ax):
    """The captured 8-iteration block replays exactly the eager iteration."""
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (3, 3, 2))
    bd = torch.from_numpy(rhs[None]).cuda()
    xg, rg = ax.cg_solve(prob, bd, rtol=1e-10, use_graph=True)
    xe, re = ax.cg_solve(prob, bd, rtol=1e-10, use_graph=False)
    assert rg["status"] == re["status"] == "AX_OK"
    assert rg["iterations"] == re["iterations"]
    assert torch.equal(xg, xe)


@pytest.mark.parametrize("kernel", ["auto", "tile", "slices"])
@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_batched_cg_union(ax, inner, kernel):
    """CG over the block-diagonal union of meshes of different order, with one batched AxLocal
    launch per step (the per-item kernels or, forced, the tile kernel over the work list or over
    mesh slices, all gathering the global vector); the oracle recomputes every mesh's residual of
    the GPU solution."""
    import torch
    from paper_2504_07042_amd import autotune
    precs = (ax.AX_FP64, ax.AX_FP32)
    saved = {(N, P): autotune.tune_get(N, ax.AX_TUNE_BATCHED, P) for N in range(1, 10) for P in precs}
    if kernel != "auto":
        for (N, P) in saved:
            autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, kernel=ax.AX_KERNEL_TILE, tile_alt=int(kernel == "slices"))
    try:
        _batched_cg_union(ax, inner)
    finally:
        for (N, P), s in saved.items():
            autotune.tune_set(N, ax.AX_TUNE_BATCHED, P, **{k: s[k] for k in autotune.KNOBS})


def _batched_cg_union(ax, inner):
    import torch
    specs = [(2, (3, 2, 2)), (3, (2, 2, 2)), (5, (2, 1, 2)), (4, (2, 2, 3))]
    meshes, parts, refs, rhss = [], [], [], []
    for q, (N, grid) in enumerate(specs):
        m = meshgen.jittered_hex(*grid, alpha=0.1, seed=40 + q)
        l2g, ng, mask = meshgen.global_numbering(*grid, N)
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        rhs, _ = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
        meshes.append((torch.from_numpy(m.verts).cuda(), ax.Basis(N)))
        parts.append((l2g, ng, mask))
        refs.append((N, D, G, l2g, ng, mask))
        rhss.append(rhs)
    l2g, ng, mask, loff, goff = meshgen.concat_numbering(parts)
    gs = ax.GatherScatter(l2g, ng, mask)
    b = np.concatenate(rhss)
    ip = ax.AX_FP64 if inner == "fp64" else ax.AX_FP32
    x, rep = ax.cg_solve_batched(meshes, gs, torch.from_numpy(b[None]).cuda(), rtol=1e-10, inner_prec=ip,
                                 inner_rtol=1e-5)
    assert rep["status"] == "AX_OK", rep
    x = x.cpu().numpy()[0]
    r2 = 0.0
    for q, (N, D, G, l2gq, ngq, maskq) in enumerate(refs):
        xq = x[goff[q]:goff[q + 1]]
        r = rhss[q] - oracle.apply_A(N, D, G, l2gq, ngq, maskq, xq)
        r2 += float(r @ r)
    assert np.sqrt(r2) / np.linalg.norm(b) <= 1e-10


@pytest.mark.parametrize("N,geom", [(1, "tri"), (3, "tri"), (7, "tri"), (11, "tri"), (15, "tri"), (4, "para"), (7, "para")])
def test_local_diag_vs_oracle(ax, N, geom):
    """Element diagonals of D^T G D with recomputed factors against the oracle's diagonal."""
    import torch
    if geom == "tri":
        m = meshgen.jittered_hex(3, 2, 2, alpha=0.15, seed=60 + N)
    else:
        m, _ = meshgen.parallelepiped_hex(2, 2, 3, seed=N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    ref = oracle.ax_diag(D, G)
    b = ax.Basis(N)
    V = torch.from_numpy(m.verts).cuda()
    if geom == "tri":
        dg = ax.local_diag(V, b, ax.AX_TRILINEAR)
    else:
        dg = ax.local_diag(ax.parallelepiped_factors(V), b, ax.AX_PARALLELEPIPED)
    err = np.abs(dg.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"[parity] local diag {geom} N={N} max rel err {err:.3e}", flush=True)
    assert err <= 1e-13


@pytest.mark.parametrize("N,grid", [(3, (3, 3, 3)), (5, (2, 3, 2))])
def test_jacobi_pcg_fp64_matches_oracle(ax, N, grid):
    """Jacobi-preconditioned CG (the Table 5-style solve) against the oracle's PCG: same
    iteration count up to rounding drift, same solution, and the oracle recomputes the residual."""
    import torch
    m, prob, ref, rhs = _problem(ax, N, grid)
    D, G, l2g, ng, mask = ref
    xg, rep = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-10, precond=ax.AX_PRECOND_JACOBI)
    assert rep["status"] == "AX_OK", rep
    x = xg.cpu().numpy()[0]
    assert _oracle_rel_res(N, ref, rhs, x) <= 1e-10
    dinv = oracle.jacobi_dinv(D, G, l2g, ng, mask)
    xo, it, rel = oracle.pcg(N, D, G, l2g, ng, mask, rhs, dinv, rtol=1e-10)
    assert np.abs(x - xo).max() <= 1e-8 * np.abs(xo).max()
    assert abs(rep["iterations"] - it) <= max(2, it // 100), (rep["iterations"], it)
    _, r_cg = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-10)
    print(f"[pcg] N={N} grid={grid} jacobi {rep['iterations']} its (oracle {it}), plain {r_cg['iterations']}", flush=True)
    assert rep["iterations"] < r_cg["iterations"]


@pytest.mark.parametrize("refine", ["reliable", "restart"])
def test_jacobi_pcg_mixed_reaches_fp64_residual(ax, refine):
    import torch
    N = 4
    m, prob, ref, rhs = _problem(ax, N, (3, 3, 3))
    kw = dict(inner_rtol=0.1, refine=ax.AX_REFINE_RELIABLE) if refine == "reliable" else dict(inner_rtol=1e-5)
    xg, rep = ax.cg_solve(prob, torch.from_numpy(rhs[None]).cuda(), rtol=1e-10, inner_prec=ax.AX_FP32,
                          precond=ax.AX_PRECOND_JACOBI, **kw)
    assert rep["status"] == "AX_OK", rep
    assert rep["outer_it"] >= 2
    assert _oracle_rel_res(N, ref, rhs, xg.cpu().numpy()[0]) <= 1e-10


def test_jacobi_pcg_graph_replay_equals_eager(ax):
    import torch
    N = 3
    m, prob, ref, rhs = _problem(ax, N, (3, 3, 2))
    bd = torch.from_numpy(rhs[None]).cuda()
    xg, rg = ax.cg_solve(prob, bd, rtol=1e-10, use_graph=True, precond=ax.AX_PRECOND_JACOBI)
    xe, re = ax.cg_solve(prob, bd, rtol=1e-10, use_graph=False, precond=ax.AX_PRECOND_JACOBI)
    assert rg["status"] == re["status"] == "AX_OK"
    assert rg["iterations"] == re["iterations"]
    assert torch.equal(xg, xe)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_jacobi_batched_cg_union(ax, inner):
    """Jacobi PCG over the block-diagonal union of meshes of different order (diagonals per mesh,
    one assembly of the union); the oracle recomputes every mesh's residual."""
    import torch
    specs = [(2, (3, 2, 2)), (3, (2, 2, 2)), (5, (2, 1, 2)), (4, (2, 2, 3))]
    meshes, parts, refs, rhss = [], [], [], []
    for q, (N, grid) in enumerate(specs):
        m = meshgen.jittered_hex(*grid, alpha=0.1, seed=40 + q)
        l2g, ng, mask = meshgen.global_numbering(*grid, N)
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        rhs, _ = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
        meshes.append((torch.from_numpy(m.verts).cuda(), ax.Basis(N)))
        parts.append((l2g, ng, mask))
        refs.append((N, D, G, l2g, ng, mask))
        rhss.append(rhs)
    l2g, ng, mask, loff, goff = meshgen.concat_numbering(parts)
    gs = ax.GatherScatter(l2g, ng, mask)
    b = np.concatenate(rhss)
    ip = ax.AX_FP64 if inner == "fp64" else ax.AX_FP32
    x, rep = ax.cg_solve_batched(meshes, gs, torch.from_numpy(b[None]).cuda(), rtol=1e-10, inner_prec=ip,
                                 inner_rtol=1e-5, precond=ax.AX_PRECOND_JACOBI)
    assert rep["status"] == "AX_OK", rep
    x = x.cpu().numpy()[0]
    r2 = 0.0
    for q, (N, D, G, l2gq, ngq, maskq) in enumerate(refs):
        xq = x[goff[q]:goff[q + 1]]
        r = rhss[q] - oracle.apply_A(N, D, G, l2gq, ngq, maskq, xq)
        r2 += float(r @ r)
    assert np.sqrt(r2) / np.linalg.norm(b) <= 1e-10
