"""GPU parity of the Helmholtz operator with merged scalar factors (Eq. 3, Sec. 4.2.1) and of its
set-up kernel, against the CPU oracle, through the C ABI.  The coefficient fields lambda0,
lambda1 are seeded positive random nodal values."""
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


def _case(N, nx=3, ny=3, nz=2, seed=0, sample=None):
    m = meshgen.jittered_hex(nx, ny, nz, alpha=0.15, seed=400 + N + seed)
    rng = np.random.default_rng(N + seed)
    NP = (N + 1) ** 3
    lam0 = rng.uniform(0.5, 2.0, (m.E, NP))
    lam1 = rng.uniform(0.0, 3.0, (m.E, NP))
    return m, lam0, lam1


def _oracle(m, N, lam0, lam1, X, sel=None):
    xi, w, D = oracle.gll(N)
    V = m.verts if sel is None else m.verts[sel]
    G, gwj, _ = oracle.geom_factors(V, N, xi, w)
    if sel is not None:
        lam0, lam1, X = lam0[sel], lam1[sel], X[:, sel]
    Y = oracle.ax_local_helmholtz(D, G, gwj, lam0, lam1, X)
    env = oracle.ax_envelope(D, G * lam0[:, None, :], X) + np.abs(lam1 * gwj)[None] * np.abs(X)
    return Y, env


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 11, 15])
def test_helmholtz_fp64(ax, N):
    m, lam0, lam1 = _case(N)
    X = meshgen.random_nodal(m.E, N, nrhs=1, seed=N)
    Yref, env = _oracle(m, N, lam0, lam1, X)
    b = ax.Basis(N)
    v = _dev(m.verts)
    L23 = ax.helmholtz_factors(v, _dev(lam0), _dev(lam1), b, ax.AX_FP64)
    Y = ax.ax_local_helmholtz(_dev(X), v, L23, b, ax.AX_FP64)
    check_fp64(Y.cpu().numpy(), Yref, env)


def test_helmholtz_factors_vs_oracle(ax):
    N = 5
    m, lam0, lam1 = _case(N)
    xi, w, _ = oracle.gll(N)
    _, gwj, _ = oracle.geom_factors(m.verts, N, xi, w)
    lam = oracle.lambda_geo(m.verts, N, xi, w)
    L23 = ax.helmholtz_factors(_dev(m.verts), _dev(lam0), _dev(lam1), ax.Basis(N)).cpu().numpy()
    ref2, ref3 = lam * lam0, gwj * lam1
    assert np.abs(L23[:, 0] - ref2).max() <= 1e-14 * np.abs(ref2).max()
    assert np.abs(L23[:, 1] - ref3).max() <= 1e-14 * np.abs(ref3).max()


@pytest.mark.parametrize("N", [3, 7])
def test_helmholtz_multi_rhs_and_fp32(ax, N):
    import torch
    m, lam0, lam1 = _case(N, 2, 2, 3, seed=1)
    b = ax.Basis(N)
    v = _dev(m.verts)
    X = meshgen.random_nodal(m.E, N, nrhs=2, seed=N + 1)
    Yref, env = _oracle(m, N, lam0, lam1, X)
    Y = ax.ax_local_helmholtz(_dev(X), v, ax.helmholtz_factors(v, _dev(lam0), _dev(lam1), b), b).cpu().numpy()
    for c in range(2):
        check_fp64(Y[c], Yref[c], env[c])
    X32 = X[:1].astype(np.float32)
    Yr32, env32 = _oracle(m, N, lam0, lam1, X32.astype(np.float64))
    L32 = ax.helmholtz_factors(v, _dev(lam0), _dev(lam1), b, ax.AX_FP32)
    Y32 = ax.ax_local_helmholtz(torch.from_numpy(X32).cuda(), v, L32, b, ax.AX_FP32)
    check_bound(Y32.cpu().numpy(), Yr32, env32, fp32_bound(N, max_cond_j(m.verts, N)))


def test_helmholtz_full_size_sampled(ax):
    """N = 7 at the benchmark's size (32^3 elements), a sample of elements against the oracle."""
    N = 7
    m = meshgen.jittered_hex(32, 32, 32, alpha=0.15, seed=N)
    rng = np.random.default_rng(3)
    NP = (N + 1) ** 3
    lam0 = rng.uniform(0.5, 2.0, (m.E, NP))
    lam1 = rng.uniform(0.0, 3.0, (m.E, NP))
    X = meshgen.random_nodal(m.E, N, seed=N)
    b = ax.Basis(N)
    v = _dev(m.verts)
    Y = ax.ax_local_helmholtz(_dev(X), v, ax.helmholtz_factors(v, _dev(lam0), _dev(lam1), b), b).cpu().numpy()
    sel = np.unique(np.concatenate([rng.choice(m.E, 61, replace=False), [0, 1, m.E - 1]]))
    Yref, env = _oracle(m, N, lam0, lam1, X, sel=sel)
    check_fp64(Y[:, sel], Yref, env)
