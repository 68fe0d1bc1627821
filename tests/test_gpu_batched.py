"""GPU batched AxLocal (one persistent launch over meshes of uneven size and order) against the
per-mesh kernel and the oracle, eagerly and replayed from a captured graph."""
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


SPECS = [(3, (3, 2, 2)), (7, (2, 2, 3)), (1, (5, 4, 3)), (5, (2, 3, 1)), (9, (2, 1, 2)), (2, (4, 4, 4)),
         (7, (1, 1, 1)), (4, (3, 3, 2)), (6, (2, 2, 2)), (8, (1, 2, 2))]


def _setup(ax, dtype, nrhs=2):
    import torch
    meshes, X, Y, host = [], [], [], []
    for q, (N, grid) in enumerate(SPECS):
        m = meshgen.jittered_hex(*grid, alpha=0.15, seed=300 + q)
        x = meshgen.random_nodal(m.E, N, nrhs=nrhs, seed=q)
        if dtype == "f32":
            x = x.astype(np.float32)
        b = ax.Basis(N)
        meshes.append((torch.from_numpy(m.verts).cuda(), b))
        X.append(torch.from_numpy(x).cuda())
        Y.append(torch.full_like(X[-1], float("nan")))
        host.append((N, m, x))
    return meshes, X, Y, host


def test_batched_fp64_matches_single_and_oracle(ax):
    import torch
    meshes, X, Y, host = _setup(ax, "f64")
    bat = ax.BatchedAxLocal(meshes, X, Y, ax.AX_FP64)
    bat.launch()
    torch.cuda.synchronize()
    for q, (N, m, x) in enumerate(host):
        Ys = ax.ax_local(X[q], meshes[q][0], meshes[q][1], ax.AX_TRILINEAR, ax.AX_FP64)
        yb = Y[q].cpu().numpy()
        assert np.allclose(yb, Ys.cpu().numpy(), rtol=0, atol=1e-14 * np.abs(yb).max())
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        check_fp64(yb, oracle.ax_local(D, G, x), oracle.ax_envelope(D, G, x))


def test_batched_fp32(ax):
    meshes, X, Y, host = _setup(ax, "f32")
    bat = ax.BatchedAxLocal(meshes, X, Y, ax.AX_FP32)
    bat.launch()
    for q, (N, m, x) in enumerate(host):
        xd = x.astype(np.float64)
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        check_bound(Y[q].cpu().numpy(), oracle.ax_local(D, G, xd), oracle.ax_envelope(D, G, xd),
                    fp32_bound(N, max_cond_j(m.verts, N)))


def test_batched_graph_replay(ax):
    """Capture the single launch in a graph; replay it several times with eager work and
    synchronisations in between; every replay must equal the eager result."""
    import torch
    meshes, X, Y, host = _setup(ax, "f64", nrhs=1)
    bat = ax.BatchedAxLocal(meshes, X, Y, ax.AX_FP64)
    bat.launch()
    torch.cuda.synchronize()
    eager = [y.clone() for y in Y]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bat.launch(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for y in Y:
            y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for q in range(len(Y)):
            assert torch.equal(Y[q], eager[q]), (rep, q)
        _ = (X[0] * 2.0).sum().item()  # unrelated eager work between replays


def test_batched_validation(ax):
    import ctypes
    p = (ax.AxProblem * 1)()
    b = ax.Basis(12)
    p[0] = ax.AxProblem(4, 12, 0, 8, b.D.ctypes.data, b.xi.ctypes.data, b.w.ctypes.data, 0, None, None, None, None)
    n = ctypes.c_size_t()
    assert ax.lib().ax_batched_workspace_bytes(1, p, ctypes.byref(n)) == ax.AX_ERR_UNSUPPORTED
