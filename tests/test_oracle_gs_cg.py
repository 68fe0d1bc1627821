"""Pins of the oracle's gather-scatter (Sec. 2.1, Eq. 1) and CG against counts printed by the
paper, sparse-matrix products (scipy) and a direct dense solve."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import dense
from conftest import golden
from paper_2504_07042_amd import meshgen


def test_fig1_counts():
    g = golden("fig1_counts.json")
    l2g, ng, mask = meshgen.chain_numbering(g["E"], g["N"])
    assert ng == g["n_global"]
    assert len(np.unique(l2g)) == g["n_global"]
    assert l2g.size == g["E"] * (g["N"] + 1) ** 3


@pytest.mark.parametrize("N", [1, 3, 4])
def test_multiplicity_classes(N):
    """Q^T 1 counts how many elements share a node: 8 at interior vertices, 4 on interior edges,
    2 on interior faces, 1 inside elements (and fewer on the boundary)."""
    nx, ny, nz = 3, 2, 4
    l2g, ng, mask = meshgen.global_numbering(nx, ny, nz, N)
    mult = oracle.gs_qt(l2g, ng, np.ones((1, l2g.size)))[0]
    assert set(np.unique(mult)) <= {1.0, 2.0, 4.0, 8.0}
    assert mult.sum() == l2g.size
    n_v = (nx - 1) * (ny - 1) * (nz - 1)
    assert np.sum(mult == 8) == n_v
    Gx, Gy, Gz = nx * N + 1, ny * N + 1, nz * N + 1
    assert ng == Gx * Gy * Gz
    assert mask.sum() == ng - (Gx - 2) * (Gy - 2) * (Gz - 2)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_element_numbering_is_a_renumbering(N):
    """The first-touch (element-major) numbering is a permutation of the lexicographic grid
    numbering that carries the Dirichlet mask along, and numbers nodes in order of first
    appearance."""
    la, ng, ma = meshgen.global_numbering(3, 2, 2, N)
    lb, ngb, mb = meshgen.global_numbering(3, 2, 2, N, order="element")
    assert ng == ngb
    perm = np.full(ng, -1, dtype=np.int64)
    perm[la] = lb
    assert np.array_equal(perm[la], lb)
    assert np.array_equal(np.sort(perm), np.arange(ng))
    assert np.array_equal(mb[perm], ma)
    _, first = np.unique(lb, return_index=True)
    assert np.all(np.diff(first) > 0)


@pytest.mark.parametrize("N", [2, 3])
def test_q_and_qt_vs_sparse(N):
    l2g, ng, _ = meshgen.global_numbering(2, 3, 2, N)
    Q = sp.csr_matrix((np.ones(l2g.size), (np.arange(l2g.size), l2g)), shape=(l2g.size, ng))
    rng = np.random.default_rng(0)
    yl = rng.uniform(-1, 1, (2, l2g.size))
    xg = rng.uniform(-1, 1, (2, ng))
    assert np.allclose(oracle.gs_qt(l2g, ng, yl), (Q.T @ yl.T).T, rtol=0, atol=1e-15)
    assert np.array_equal(oracle.gs_q(l2g, xg), (Q @ xg.T).T)
    QtQ = (Q.T @ Q).toarray()
    mult = oracle.gs_qt(l2g, ng, np.ones((1, l2g.size)))[0]
    assert np.array_equal(QtQ, np.diag(mult))


def test_qt_sums_in_ascending_local_order():
    """Q^T adds contributions in ascending local index: check with values whose floating-point
    sum depends on the order."""
    l2g = np.array([0, 1, 0, 0], dtype=np.int32)
    y = np.array([[1e16, 5.0, 1.0, -1e16]])
    out = oracle.gs_qt(l2g, 2, y)[0]
    assert out[0] == ((1e16 + 1.0) + -1e16)
    assert out[1] == 5.0


@pytest.mark.parametrize("N", [2, 3])
def test_apply_a_matches_dense_assembly(N):
    m = meshgen.jittered_hex(2, 2, 2, alpha=0.1, seed=4)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(2, 2, 2, N)
    A = dense.assembled_matrix(D, G, l2g, ng, mask)
    x = np.random.default_rng(2).uniform(-1, 1, ng)
    x[mask == 1] = 0
    y = oracle.apply_A(N, D, G, l2g, ng, mask, x)
    assert np.allclose(y, A @ x, rtol=0, atol=1e-13 * np.abs(A).max())


def test_cg_matches_direct_solve():
    N = 3
    m = meshgen.jittered_hex(3, 3, 3, alpha=0.1, seed=4)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(3, 3, 3, N)
    b, _ = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
    x, it, rel = oracle.cg(N, D, G, l2g, ng, mask, b, rtol=1e-12)
    assert it > 0 and rel <= 1e-11
    A = dense.assembled_matrix(D, G, l2g, ng, mask)
    free = mask == 0
    xd = np.zeros(ng)
    xd[free] = np.linalg.solve(A[np.ix_(free, free)], b[free])
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()


def test_cg_manufactured_solution():
    """-Lap u = 3 pi^2 u for u = sin(pi x) sin(pi y) sin(pi z): the discrete solution converges to
    the nodal values of u (spectral accuracy; N = 5 on a 3^3 jittered mesh)."""
    N = 5
    m = meshgen.jittered_hex(3, 3, 3, alpha=0.1, seed=4)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(3, 3, 3, N)
    b, u_nodes = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
    x, it, rel = oracle.cg(N, D, G, l2g, ng, mask, b, rtol=1e-10)
    assert rel <= 1e-10
    ug = np.zeros(ng)
    ug[l2g] = u_nodes.reshape(-1)
    assert np.abs(x - ug).max() < 2e-3


def test_cg_breakdown_on_nan():
    N = 2
    m = meshgen.jittered_hex(2, 2, 2, alpha=0.0)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(2, 2, 2, N)
    b = np.ones(ng)
    b[mask == 1] = 0
    b[ng // 2] = np.nan
    _, it, _ = oracle.cg(N, D, G, l2g, ng, mask, b)
    assert it == -1


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_element_diagonal_vs_dense(N):
    """The element diagonal is the diagonal of the brute-force Kronecker element matrix."""
    m = meshgen.jittered_hex(2, 1, 2, alpha=0.2, seed=30 + N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    dg = oracle.ax_diag(D, G)
    for e in range(m.E):
        ref = np.diag(dense.element_matrix(D, G[e]))
        assert np.abs(dg[e] - ref).max() <= 1e-13 * np.abs(ref).max()
        assert (dg[e] > 0).all()


@pytest.mark.parametrize("N", [2, 3])
def test_jacobi_inverse_vs_dense_assembly(N):
    """Q^T of the element diagonals is the diagonal of the assembled operator (Eq. 1) on the free
    nodes; the inverse is zero on the Dirichlet nodes."""
    m = meshgen.jittered_hex(2, 2, 2, alpha=0.15, seed=40 + N)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(2, 2, 2, N)
    dinv = oracle.jacobi_dinv(D, G, l2g, ng, mask)
    A = dense.assembled_matrix(D, G, l2g, ng, mask)
    free = mask == 0
    assert np.abs(dinv[free] * np.diag(A)[free] - 1.0).max() <= 1e-13
    assert (dinv[~free] == 0).all()


def test_pcg_matches_direct_solve_in_fewer_iterations():
    N = 3
    m = meshgen.jittered_hex(3, 3, 3, alpha=0.1, seed=4)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(3, 3, 3, N)
    b, _ = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
    dinv = oracle.jacobi_dinv(D, G, l2g, ng, mask)
    x, it, rel = oracle.pcg(N, D, G, l2g, ng, mask, b, dinv, rtol=1e-12)
    assert it > 0 and rel <= 1e-11
    A = dense.assembled_matrix(D, G, l2g, ng, mask)
    free = mask == 0
    xd = np.zeros(ng)
    xd[free] = np.linalg.solve(A[np.ix_(free, free)], b[free])
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()
    _, it_cg, _ = oracle.cg(N, D, G, l2g, ng, mask, b, rtol=1e-12)
    assert it < it_cg


def test_pcg_with_identity_is_cg():
    """With M = I on the free nodes the preconditioned recurrence is plain CG's: same iteration
    count and the same iterate up to rounding."""
    N = 2
    m = meshgen.jittered_hex(2, 2, 3, alpha=0.1, seed=8)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    l2g, ng, mask = meshgen.global_numbering(2, 2, 3, N)
    b, _ = oracle.poisson_rhs(N, m.verts, xi, w, l2g, ng, mask)
    one = np.where(mask == 1, 0.0, 1.0)
    x1, it1, _ = oracle.pcg(N, D, G, l2g, ng, mask, b, one, rtol=1e-10)
    x0, it0, _ = oracle.cg(N, D, G, l2g, ng, mask, b, rtol=1e-10)
    assert it1 == it0
    assert np.abs(x1 - x0).max() <= 1e-12 * np.abs(x0).max()
