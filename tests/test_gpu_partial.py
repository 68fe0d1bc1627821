"""GPU parity of the partial-recomputation operator (Sec. 4.2.2: the per-node scale read from
memory, K and adj(K) recomputed) and of its set-up kernel, against the CPU oracle, through the
C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import check_bound, check_fp64, fp32_bound, max_cond_j
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


@pytest.mark.parametrize("N", [1, 2, 3, 7, 10, 15])
def test_lambda_setup_vs_oracle(ax, N):
    m = meshgen.jittered_hex(3, 3, 2, alpha=0.15, seed=300 + N)
    xi, w, _ = oracle.gll(N)
    ref = oracle.lambda_geo(m.verts, N, xi, w)
    lam = ax.geom_lambda(_dev(m.verts), ax.Basis(N), ax.AX_FP64).cpu().numpy()
    assert np.abs(lam - ref).max() <= 1e-14 * np.abs(ref).max()
    lam32 = ax.geom_lambda(_dev(m.verts), ax.Basis(N), ax.AX_FP32).cpu().numpy()
    assert lam32.dtype == np.float32
    assert np.abs(lam32 - ref).max() <= 2.0**-23 * np.abs(ref).max()


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_partial_fp64(ax, N):
    # 18 elements: a ragged last work-group for every elements-per-group choice
    m = meshgen.jittered_hex(3, 3, 2, alpha=0.15, seed=100 + N)
    X = meshgen.random_nodal(m.E, N, nrhs=1, seed=N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Yref, env = oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X)
    b = ax.Basis(N)
    v = _dev(m.verts)
    lam = ax.geom_lambda(v, b, ax.AX_FP64)
    Y = ax.ax_local_partial(_dev(X), v, lam, b, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


@pytest.mark.parametrize("N", [3, 7])
def test_partial_multi_rhs(ax, N):
    m = meshgen.jittered_hex(2, 3, 2, alpha=0.15, seed=7 + N)
    X = meshgen.random_nodal(m.E, N, nrhs=3, seed=N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    b = ax.Basis(N)
    v = _dev(m.verts)
    Y = ax.ax_local_partial(_dev(X), v, ax.geom_lambda(v, b), b).cpu().numpy()
    for c in range(3):
        check_fp64(Y[c], oracle.ax_local(D, G, X[c:c + 1])[0], oracle.ax_envelope(D, G, X[c:c + 1])[0])


@pytest.mark.parametrize("N", [1, 3, 7, 11, 12, 13, 14])
def test_partial_fp32(ax, N):
    import torch
    m = meshgen.jittered_hex(3, 2, 2, alpha=0.15, seed=200 + N)
    X32 = meshgen.random_nodal(m.E, N, seed=N).astype(np.float32)
    X = X32.astype(np.float64)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Yref, env = oracle.ax_local(D, G, X), oracle.ax_envelope(D, G, X)
    b = ax.Basis(N)
    v = _dev(m.verts)
    Y = ax.ax_local_partial(torch.from_numpy(X32).cuda(), v, ax.geom_lambda(v, b, ax.AX_FP32), b, ax.AX_FP32)
    check_bound(Y.cpu().numpy(), Yref, env, fp32_bound(N, max_cond_j(m.verts, N)))


def test_partial_full_size_sampled(ax):
    """N = 7 at the benchmark's size (32^3 elements), a sample of elements against the oracle."""
    N = 7
    m = meshgen.jittered_hex(32, 32, 32, alpha=0.15, seed=N)
    X = meshgen.random_nodal(m.E, N, seed=N)
    b = ax.Basis(N)
    v = _dev(m.verts)
    Y = ax.ax_local_partial(_dev(X), v, ax.geom_lambda(v, b), b).cpu().numpy()
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([rng.choice(m.E, 61, replace=False), [0, 1, m.E - 1]]))
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts[sample], N, xi, w)
    Xs = X[:, sample]
    check_fp64(Y[:, sample], oracle.ax_local(D, G, Xs), oracle.ax_envelope(D, G, Xs))


def test_partial_empty_mesh_is_noop(ax):
    import torch
    b = ax.Basis(3)
    X = torch.zeros((1, 0, 64), dtype=torch.float64, device="cuda")
    verts = torch.zeros((0, 8, 3), dtype=torch.float64, device="cuda")
    lam = torch.zeros((0, 64), dtype=torch.float64, device="cuda")
    assert ax.ax_local_partial(X, verts, lam, b).numel() == 0
