"""Full-size parity: every order of the trilinear order sweep at its benchmark size
(E (N+1)^3 ~ 2^24 local nodes, +-15 % jitter, seed N), in FP64 and FP32, for the on-the-fly,
partial-recomputation and stored-factor operators, plus parallelepipeds and a strongly
distorted mesh.  The library runs the whole mesh in the same launch configuration the
benchmark times (persistent work-groups that take many element groups each); a seeded sample
of elements (first, last, ragged tail, random) is compared with the oracle element by element,
which is exact because AxLocal is element-local.  Every check prints its observed ratio."""
import numpy as np
import pytest

import oracle
from gpu_util import (check_bound, check_fp64, cond_j_per_element, fp32_bound, report,
                      sample_elements)
from paper_2504_07042_amd import meshgen

pytestmark = pytest.mark.gpu

SWEEP = [3, 5, 7, 9, 11, 15]
_CACHE = {}


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_07042_amd as ax
    ax.lib()
    return ax


def _case(ax, N):
    """Mesh, nodal X, device copies and the oracle's reference on the sample, for order N."""
    import torch
    if N in _CACHE:
        return _CACHE[N]
    _CACHE.clear()
    torch.cuda.empty_cache()
    grid = meshgen.grid_for_nodes(N)
    m = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
    X = meshgen.random_nodal(m.E, N, seed=N)
    sample = sample_elements(m.E, seed=N)
    xi, w, D = oracle.gll(N)
    G, _, mind = oracle.geom_factors(m.verts[sample], N, xi, w)
    assert mind > 0
    X32 = X.astype(np.float32)
    c = {
        "m": m, "sample": sample, "D": D, "G": G,
        "V": torch.from_numpy(m.verts).cuda(),
        "X64": torch.from_numpy(X).cuda(),
        "X32": torch.from_numpy(X32).cuda(),
        "Yref64": oracle.ax_local(D, G, X[:, sample]),
        "env64": oracle.ax_envelope(D, G, X[:, sample]),
        "Yref32": oracle.ax_local(D, G, X32[:, sample].astype(np.float64)),
        "env32": oracle.ax_envelope(D, G, X32[:, sample].astype(np.float64)),
        "kappa": cond_j_per_element(m.verts[sample], N)[None, :, None],
        "b": ax.Basis(N),
    }
    print(f"[fullsize] N={N} grid={grid} E={m.E} local nodes={m.E * (N + 1) ** 3} "
          f"sample={len(sample)} max kappa_J={c['kappa'].max():.2f}", flush=True)
    _CACHE[N] = c
    return c


def _sampled(Y, sample):
    import torch
    idx = torch.from_numpy(sample).cuda()
    return Y.index_select(1, idx).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("N", SWEEP)
def test_sweep_on_the_fly_fp64(ax, N):
    c = _case(ax, N)
    Y = ax.ax_local(c["X64"], c["V"], c["b"], ax.AX_TRILINEAR, ax.AX_FP64)
    check_fp64(_sampled(Y, c["sample"]), c["Yref64"], c["env64"], tag=f"fullsize on-the-fly fp64 N={N}")


@pytest.mark.parametrize("N", SWEEP)
def test_sweep_on_the_fly_fp32(ax, N):
    c = _case(ax, N)
    Y = ax.ax_local(c["X32"], c["V"], c["b"], ax.AX_TRILINEAR, ax.AX_FP32)
    check_bound(_sampled(Y, c["sample"]), c["Yref32"], c["env32"], fp32_bound(N, c["kappa"]),
                tag=f"fullsize on-the-fly fp32 N={N}")


@pytest.mark.parametrize("N", SWEEP)
def test_sweep_partial_fp64(ax, N):
    c = _case(ax, N)
    lam = ax.geom_lambda(c["V"], c["b"], ax.AX_FP64)
    Y = ax.ax_local_partial(c["X64"], c["V"], lam, c["b"], ax.AX_FP64)
    check_fp64(_sampled(Y, c["sample"]), c["Yref64"], c["env64"], tag=f"fullsize partial fp64 N={N}")


@pytest.mark.parametrize("N", SWEEP)
def test_sweep_partial_fp32(ax, N):
    c = _case(ax, N)
    lam = ax.geom_lambda(c["V"], c["b"], ax.AX_FP32)
    Y = ax.ax_local_partial(c["X32"], c["V"], lam, c["b"], ax.AX_FP32)
    check_bound(_sampled(Y, c["sample"]), c["Yref32"], c["env32"], fp32_bound(N, c["kappa"]),
                tag=f"fullsize partial fp32 N={N}")


@pytest.mark.parametrize("N", SWEEP)
def test_sweep_stored_fp64(ax, N):
    c = _case(ax, N)
    G, _ = ax.geom_factors(c["V"], c["b"], ax.AX_FP64)
    Y = ax.ax_local_precomputedG(c["X64"], G, c["b"], ax.AX_FP64)
    del G
    check_fp64(_sampled(Y, c["sample"]), c["Yref64"], c["env64"], tag=f"fullsize stored fp64 N={N}")


@pytest.mark.parametrize("N", [3, 7])
def test_stored_fp32_full_size(ax, N):
    c = _case(ax, N)
    G, _ = ax.geom_factors(c["V"], c["b"], ax.AX_FP32)
    Y = ax.ax_local_precomputedG(c["X32"], G, c["b"], ax.AX_FP32)
    del G
    check_bound(_sampled(Y, c["sample"]), c["Yref32"], c["env32"], fp32_bound(N, c["kappa"]),
                tag=f"fullsize stored fp32 N={N}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_parallelepiped_full_size(ax, prec):
    """N = 7 on the 32^3 sheared cube (every element the same parallelepiped, cond <= 4)."""
    import torch
    N = 7
    m, _ = meshgen.parallelepiped_hex(32, 32, 32, seed=2)
    X = meshgen.random_nodal(m.E, N, seed=N + 50)
    if prec == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    sample = sample_elements(m.E, seed=2)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts[sample], N, xi, w)
    b = ax.Basis(N)
    h = ax.parallelepiped_factors(torch.from_numpy(m.verts).cuda())
    if prec == "fp64":
        Y = ax.ax_local(torch.from_numpy(X).cuda(), h, b, ax.AX_PARALLELEPIPED, ax.AX_FP64)
        check_fp64(_sampled(Y, sample), oracle.ax_local(D, G, X[:, sample]),
                   oracle.ax_envelope(D, G, X[:, sample]), tag="fullsize parallelepiped fp64 N=7")
    else:
        kappa = cond_j_per_element(m.verts[sample[:4]], N).max()
        Y = ax.ax_local(torch.from_numpy(X.astype(np.float32)).cuda(), h, b, ax.AX_PARALLELEPIPED, ax.AX_FP32)
        check_bound(_sampled(Y, sample), oracle.ax_local(D, G, X[:, sample]),
                    oracle.ax_envelope(D, G, X[:, sample]), fp32_bound(N, kappa),
                    tag="fullsize parallelepiped fp32 N=7")


# Strongly distorted meshes: interior vertices jittered by 38 % (5x5x4) and 30 % (8^3) of h,
# seeds picked so that det J > 0 at every GLL node (independent per-coordinate jitter of
# 35-40 % inverts some element of any larger box); the Jacobians reach cond ~ 10^2.
DISTORTED = {"a38": ((5, 5, 4), 0.38, 45), "a30": ((8, 8, 8), 0.30, 21)}


@pytest.mark.parametrize("name", list(DISTORTED))
@pytest.mark.parametrize("N", [3, 7, 15])
def test_distorted_mesh(ax, name, N):
    import torch
    grid, alpha, seed = DISTORTED[name]
    m = meshgen.jittered_hex(*grid, alpha=alpha, seed=seed)
    xi, w, D = oracle.gll(N)
    G, _, mind = oracle.geom_factors(m.verts, N, xi, w)
    assert mind > 0, "the distorted mesh must stay valid (det J > 0 at every node)"
    kappa = cond_j_per_element(m.verts, N)
    report(f"distorted {name} N={N}", E=m.E, min_detJ=float(mind), max_kappa_J=float(kappa.max()))
    X = meshgen.random_nodal(m.E, N, nrhs=2, seed=seed)
    b = ax.Basis(N)
    V = torch.from_numpy(m.verts).cuda()
    Y = ax.ax_local(torch.from_numpy(X).cuda(), V, b, ax.AX_TRILINEAR, ax.AX_FP64).cpu().numpy()
    check_fp64(Y, oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X), tag=f"distorted {name} fp64 N={N}")
    lam = ax.geom_lambda(V, b, ax.AX_FP64)
    Y = ax.ax_local_partial(torch.from_numpy(X).cuda(), V, lam, b, ax.AX_FP64).cpu().numpy()
    check_fp64(Y, oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X),
               tag=f"distorted {name} partial fp64 N={N}")
    X32 = X.astype(np.float32)
    Xr = X32.astype(np.float64)
    Y = ax.ax_local(torch.from_numpy(X32).cuda(), V, b, ax.AX_TRILINEAR, ax.AX_FP32).cpu().numpy()
    check_bound(Y, oracle.ax_local(D, G, Xr), oracle.ax_envelope(D, G, Xr),
                fp32_bound(N, kappa[None, :, None]), tag=f"distorted {name} fp32 N={N}")
