"""GPU parity of AxLocal (all geometries, orders, precisions) against the CPU oracle, called
through the C ABI.  Inputs are seeded synthetic meshes; the oracle computes every expected
value from the same input arrays."""
import numpy as np
import pytest

import oracle
from gpu_util import check_bound, check_fp64, fp32_bound, max_cond_j, report
from paper_2504_07042_amd import meshgen

pytestmark = pytest.mark.gpu

ALL_N = list(range(1, 16))


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


def _oracle_ref(mesh, N, X):
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(mesh.verts, N, xi, w)
    return oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X), G


def _mesh_for(N):
    # element counts that leave a ragged last work-group for every elements-per-group choice
    return meshgen.jittered_hex(3, 3, 2, alpha=0.15, seed=100 + N)


@pytest.mark.parametrize("N", ALL_N)
def test_trilinear_fp64(ax, N):
    m = _mesh_for(N)
    X = meshgen.random_nodal(m.E, N, nrhs=1, seed=N)
    Yref, env, _ = _oracle_ref(m, N, X)
    b = ax.Basis(N)
    Y = ax.ax_local(_dev(X), _dev(m.verts), b, ax.AX_TRILINEAR, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


@pytest.mark.parametrize("N", ALL_N)
def test_parallelepiped_fp64(ax, N):
    mesh, _ = meshgen.parallelepiped_hex(3, 2, 3, seed=N)
    X = meshgen.random_nodal(mesh.E, N, nrhs=1, seed=N + 50)
    Yref, env, _ = _oracle_ref(mesh, N, X)
    b = ax.Basis(N)
    verts = _dev(mesh.verts)
    h = ax.parallelepiped_factors(verts)
    hr = oracle.parallelepiped_h(mesh.verts)
    assert np.abs(h.cpu().numpy() - hr).max() <= 1e-14 * np.abs(hr).max()
    Y = ax.ax_local(_dev(X), h, b, ax.AX_PARALLELEPIPED, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


@pytest.mark.parametrize("N", ALL_N)
def test_stored_factors_fp64(ax, N):
    """Set-up kernel G vs the oracle's Eq. (7) (Frobenius relative per element <= 1e-14), then
    the stored-factor operator vs the oracle."""
    m = _mesh_for(N)
    X = meshgen.random_nodal(m.E, N, nrhs=1, seed=N + 7)
    Yref, env, Gref = _oracle_ref(m, N, X)
    b = ax.Basis(N)
    G, gwj = ax.geom_factors(_dev(m.verts), b, ax.AX_FP64, want_gwj=True)
    Gg = G.cpu().numpy()
    rel = np.linalg.norm((Gg - Gref).reshape(m.E, -1), axis=1) / np.linalg.norm(Gref.reshape(m.E, -1), axis=1)
    assert rel.max() <= 1e-14, rel.max()
    xi, w, _ = oracle.gll(N)
    _, gwj_ref, _ = oracle.geom_factors(m.verts, N, xi, w)
    assert np.abs(gwj.cpu().numpy() - gwj_ref).max() <= 1e-14 * np.abs(gwj_ref).max()
    Y = ax.ax_local_precomputedG(_dev(X), G, b, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


@pytest.mark.parametrize("N", [1, 3, 7, 8, 15])
def test_multi_rhs(ax, N):
    m = meshgen.jittered_hex(2, 3, 2, alpha=0.1, seed=N)
    X = meshgen.random_nodal(m.E, N, nrhs=3, seed=N)
    Yref, env, _ = _oracle_ref(m, N, X)
    b = ax.Basis(N)
    Y = ax.ax_local(_dev(X), _dev(m.verts), b, ax.AX_TRILINEAR, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


@pytest.mark.parametrize("N", [1, 3, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15])
def test_trilinear_fp32(ax, N):
    import torch
    m = meshgen.jittered_hex(3, 2, 2, alpha=0.15, seed=200 + N)
    X32 = meshgen.random_nodal(m.E, N, seed=N).astype(np.float32)
    X = X32.astype(np.float64)
    Yref, env, _ = _oracle_ref(m, N, X)
    b = ax.Basis(N)
    Y = ax.ax_local(torch.from_numpy(X32).cuda(), _dev(m.verts), b, ax.AX_TRILINEAR, ax.AX_FP32)
    kappa = max_cond_j(m.verts, N)
    check_bound(Y.cpu().numpy(), Yref, env, fp32_bound(N, kappa))


@pytest.mark.parametrize("N", [3, 7])
def test_parallelepiped_and_stored_fp32(ax, N):
    import torch
    mesh, _ = meshgen.parallelepiped_hex(2, 2, 3, seed=N)
    X32 = meshgen.random_nodal(mesh.E, N, seed=N).astype(np.float32)
    X = X32.astype(np.float64)
    Yref, env, _ = _oracle_ref(mesh, N, X)
    b = ax.Basis(N)
    verts = _dev(mesh.verts)
    kappa = max_cond_j(mesh.verts, N)
    h = ax.parallelepiped_factors(verts)
    Y = ax.ax_local(torch.from_numpy(X32).cuda(), h, b, ax.AX_PARALLELEPIPED, ax.AX_FP32)
    check_bound(Y.cpu().numpy(), Yref, env, fp32_bound(N, kappa))
    G32, _ = ax.geom_factors(verts, b, ax.AX_FP32)
    Y = ax.ax_local_precomputedG(torch.from_numpy(X32).cuda(), G32, b, ax.AX_FP32)
    check_bound(Y.cpu().numpy(), Yref, env, fp32_bound(N, kappa))


def test_empty_mesh_is_noop(ax):
    import torch
    b = ax.Basis(3)
    X = torch.zeros((1, 0, 64), dtype=torch.float64, device="cuda")
    verts = torch.zeros((0, 8, 3), dtype=torch.float64, device="cuda")
    Y = ax.ax_local(X, verts, b)
    assert Y.numel() == 0


def test_deterministic(ax):
    m = meshgen.jittered_hex(4, 4, 4, alpha=0.15, seed=3)
    X = _dev(meshgen.random_nodal(m.E, 7, seed=3))
    b = ax.Basis(7)
    v = _dev(m.verts)
    Y1 = ax.ax_local(X, v, b).cpu().numpy()
    Y2 = ax.ax_local(X, v, b).cpu().numpy()
    assert np.array_equal(Y1, Y2)


@pytest.mark.parametrize("N,geom", [(7, "tri"), (7, "para"), (3, "tri"), (9, "tri"), (11, "para")])
def test_full_size_sampled(ax, N, geom):
    """At the benchmark's full size (about 2^24 local nodes, same launch as the benchmark),
    compare a random sample of elements with the oracle (AxLocal is element-local)."""
    nx, ny, nz = meshgen.grid_for_nodes(N)
    if geom == "tri":
        m = meshgen.jittered_hex(nx, ny, nz, alpha=0.15, seed=N)
    else:
        m, _ = meshgen.parallelepiped_hex(nx, ny, nz, seed=2)
    X = meshgen.random_nodal(m.E, N, seed=N)
    b = ax.Basis(N)
    v = _dev(m.verts)
    if geom == "tri":
        Y = ax.ax_local(_dev(X), v, b, ax.AX_TRILINEAR, ax.AX_FP64)
    else:
        Y = ax.ax_local(_dev(X), ax.parallelepiped_factors(v), b, ax.AX_PARALLELEPIPED, ax.AX_FP64)
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([rng.choice(m.E, 61, replace=False), [0, 1, m.E - 1]]))
    sub = meshgen.HexMesh(len(sample), 1, 1, m.verts[sample])
    Yref, env, _ = _oracle_ref(sub, N, X[:, sample])
    check_fp64(Y.cpu().numpy()[:, sample], Yref, env)


def _fp16_bound(N, kappa, D, G, X, env, envmax):
    """Entrywise bound of the half-precision operator (csrc/ax_local_f16.hip), derived from its
    arithmetic: X, D, r/s/t and D^T are each rounded to half once (4 u16 relative on the
    envelope), the rest is the FP32 kernel's arithmetic, and two absolute terms cover values that
    land in half's subnormal range (absolute spacing 2^-24) after the per-element power-of-two
    scaling: X is scaled by 2^-ex with 2^ex <= 2 max|X_e|, so each rounded entry errs by at most
    2^-25 2^ex <= 2^-24 max|X_e| (propagated by the operator: 2^-24 env(max|X_e| 1)); r, s, t are
    scaled likewise by their maximum M_R <= 3 g_max ||D||_inf max|X_e| and pass through D^T in
    three directions, adding at most 9 2^-24 ||D||_1 ||D||_inf g_max max|X_e| per output entry."""
    u16 = 2.0**-11
    mx = np.abs(X).max(axis=2, keepdims=True)                      # [nrhs][E][1]
    gmax = np.abs(G).max(axis=(1, 2))[None, :, None]               # [1][E][1]
    d1 = np.abs(D).sum(axis=0).max()                               # ||D||_1
    dinf = np.abs(D).sum(axis=1).max()                             # ||D||_inf
    return ((4 * u16 + fp32_bound(N, kappa)) * env + 2.0**-24 * envmax
            + 9 * 2.0**-24 * d1 * dinf * gmax * mx)


@pytest.mark.parametrize("geom", ["tri", "para", "stored"])
def test_fp16_mfma(ax, geom):
    import torch
    N = 7
    if geom == "para":
        m, _ = meshgen.parallelepiped_hex(3, 2, 2, seed=5)
    else:
        m = meshgen.jittered_hex(3, 2, 2, alpha=0.15, seed=21)
    X32 = meshgen.random_nodal(m.E, N, nrhs=2, seed=3).astype(np.float32)
    X = X32.astype(np.float64)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Yref = oracle.ax_local(D, G, X)
    env = oracle.ax_envelope(D, G, X)
    Xmax = np.abs(X).max(axis=2, keepdims=True) * np.ones_like(X)
    envmax = oracle.ax_envelope(D, G, Xmax)
    b = ax.Basis(N)
    v = _dev(m.verts)
    Xd = torch.from_numpy(X32).cuda()
    if geom == "tri":
        Y = ax.ax_local(Xd, v, b, ax.AX_TRILINEAR, ax.AX_FP16_ACC32)
    elif geom == "para":
        Y = ax.ax_local(Xd, ax.parallelepiped_factors(v), b, ax.AX_PARALLELEPIPED, ax.AX_FP16_ACC32)
    else:
        G32, _ = ax.geom_factors(v, b, ax.AX_FP32)
        Y = ax.ax_local_precomputedG(Xd, G32, b, ax.AX_FP16_ACC32)
    kappa = max_cond_j(m.verts, N)
    d = np.abs(Y.cpu().numpy().astype(np.float64) - Yref)
    bound = _fp16_bound(N, kappa, D, G, X, env, envmax)
    report(f"fp16 {geom} N={N}", max_err_over_env=float((d / env).max()),
           max_fraction_of_bound=float((d / bound).max()))
    assert np.all(d <= bound), float((d / bound).max())
    # and it is genuinely half precision: clearly worse than the FP32 kernel would be
    assert np.linalg.norm(d) / np.linalg.norm(Yref) < 1e-2


def test_fp16_other_orders_unsupported(ax):
    import torch
    b = ax.Basis(5)
    m = meshgen.jittered_hex(1, 1, 1)
    X = torch.zeros((1, 1, 216), dtype=torch.float32, device="cuda")
    with pytest.raises(ax.AxError) as ei:
        ax.ax_local(X, _dev(m.verts), b, ax.AX_TRILINEAR, ax.AX_FP16_ACC32)
    assert ei.value.code == ax.AX_ERR_UNSUPPORTED


