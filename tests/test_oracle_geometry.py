"""Pins of the oracle's geometry: trilinear map (Eq. 8), Jacobian (Eq. 5, 9) and geometric
factors (Eq. 7), against closed forms, an independent interpolator, the factored form of
Eq. (12) and invariances."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
from paper_2504_07042_amd import meshgen


def _interp_map(V):
    """Trilinear map of one element by scipy's linear interpolation on the 2x2x2 vertex grid
    (tensor vertex order v = a + 2b + 4c <-> corner (r, s, t) = (2a-1, 2b-1, 2c-1))."""
    vals = np.empty((2, 2, 2, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                vals[a, b, c] = V[a + 2 * b + 4 * c]
    return RegularGridInterpolator(([-1.0, 1.0], [-1.0, 1.0], [-1.0, 1.0]), vals, method="linear")


def _fd_jacobian(V, r, s, t, h=0.25):
    f = _interp_map(V)
    J = np.zeros((3, 3))
    p = np.array([r, s, t])
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        a = np.clip(p + e, -1, 1)
        b = np.clip(p - e, -1, 1)
        # the map is linear along each reference axis, so the difference quotient is exact
        J[:, d] = (f(a)[0] - f(b)[0]) / (a[d] - b[d])
    return J


def _adj(K):
    return np.array([
        [K[1, 1] * K[2, 2] - K[1, 2] * K[2, 1], K[0, 2] * K[2, 1] - K[0, 1] * K[2, 2], K[0, 1] * K[1, 2] - K[0, 2] * K[1, 1]],
        [K[1, 2] * K[2, 0] - K[1, 0] * K[2, 2], K[0, 0] * K[2, 2] - K[0, 2] * K[2, 0], K[0, 2] * K[1, 0] - K[0, 0] * K[1, 2]],
        [K[1, 0] * K[2, 1] - K[1, 1] * K[2, 0], K[0, 1] * K[2, 0] - K[0, 0] * K[2, 1], K[0, 0] * K[1, 1] - K[0, 1] * K[1, 0]],
    ])


def _sym6(M):
    return np.array([M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]])


@pytest.fixture(scope="module")
def jmesh():
    return meshgen.jittered_hex(3, 2, 2, alpha=0.15, seed=11)


def test_jacobian_vs_interpolator(jmesh):
    rng = np.random.default_rng(5)
    for e in range(jmesh.E):
        V = jmesh.verts[e]
        for _ in range(4):
            r, s, t = rng.uniform(-0.9, 0.9, 3)
            J = oracle.jacobian(V, r, s, t)
            Jfd = _fd_jacobian(V, r, s, t)
            assert np.allclose(J, Jfd, rtol=0, atol=1e-13)


def test_jacobian_affine_closed_form():
    mesh, M = meshgen.parallelepiped_hex(3, 4, 5, seed=2)
    h = np.array([1 / 3, 1 / 4, 1 / 5])
    Jref = M @ np.diag(h / 2)
    for e in (0, 7, mesh.E - 1):
        for (r, s, t) in [(0, 0, 0), (-1, 1, 0.3), (0.5, -0.25, 1)]:
            assert np.allclose(oracle.jacobian(mesh.verts[e], r, s, t), Jref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_box_closed_form(N):
    """Axis-aligned box: g00 = W hy hz / (2 hx), g11 = W hx hz / (2 hy), g22 = W hx hy / (2 hz),
    off-diagonals 0, gwj = W hx hy hz / 8."""
    hx, hy, hz = 0.3, 0.7, 1.9
    V = meshgen.box_element(hx, hy, hz, origin=(0.1, -2.0, 5.0))
    xi, w, _ = oracle.gll(N)
    G, gwj, mind = oracle.geom_factors(V, N, xi, w)
    N1 = N + 1
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    assert np.allclose(G[0, 0], W * hy * hz / (2 * hx), rtol=1e-13, atol=0)
    assert np.allclose(G[0, 3], W * hx * hz / (2 * hy), rtol=1e-13, atol=0)
    assert np.allclose(G[0, 5], W * hx * hy / (2 * hz), rtol=1e-13, atol=0)
    # off-diagonals vanish up to the rounding of the vertex sums in Eq. (9)
    assert np.abs(G[0, [1, 2, 4]]).max() <= 1e-15 * np.abs(G[0, [0, 3, 5]]).max()
    assert np.allclose(gwj[0], W * hx * hy * hz / 8, rtol=1e-13, atol=0)
    assert mind == pytest.approx(hx * hy * hz / 8, rel=1e-13)
    assert G.shape == (1, 6, N1**3)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_factors_match_adjugate_form(N, jmesh):
    """Eq. (12): det J J^-1 J^-T = adj(J^T J) / det J, with J from the independent interpolator."""
    xi, w, _ = oracle.gll(N)
    G, gwj, _ = oracle.geom_factors(jmesh.verts, N, xi, w)
    N1 = N + 1
    for e in (0, jmesh.E // 2, jmesh.E - 1):
        for (i, j, k) in [(0, 0, 0), (1, N, 0), (N, 1, N - 1), (N // 2, N // 2, N // 2)]:
            l = i + j * N1 + k * N1 * N1
            J = _fd_jacobian(jmesh.verts[e], xi[i], xi[j], xi[k])
            d = np.linalg.det(J)
            W = w[i] * w[j] * w[k]
            ref = W * _sym6(_adj(J.T @ J)) / d
            scale = np.abs(ref).max()
            assert np.allclose(G[e, :, l], ref, rtol=0, atol=2e-14 * scale)
            assert gwj[e, l] == pytest.approx(W * d, rel=1e-13)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_lambda_box_closed_form(N):
    """Partial-recomputation scale on an axis-aligned box: det J = hx hy hz / 8, so
    lam = 0.125 W / det(8J) = W / (512 hx hy hz)."""
    hx, hy, hz = 0.3, 0.7, 1.9
    V = meshgen.box_element(hx, hy, hz, origin=(0.1, -2.0, 5.0))
    xi, w, _ = oracle.gll(N)
    lam = oracle.lambda_geo(V, N, xi, w)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    assert np.allclose(lam[0], W / (512 * hx * hy * hz), rtol=1e-13, atol=0)


@pytest.mark.parametrize("N", [2, 5])
def test_lambda_times_adjugate_is_factors(N, jmesh):
    """Eq. (12) in the scaling of Algorithm 2: lam * adj((8J)^T (8J)) = G, with J from the
    independent interpolator (a wrong factor 0.125 or 8 in lam fails here)."""
    xi, w, _ = oracle.gll(N)
    G, _, _ = oracle.geom_factors(jmesh.verts, N, xi, w)
    lam = oracle.lambda_geo(jmesh.verts, N, xi, w)
    N1 = N + 1
    for e in (0, jmesh.E - 1):
        for (i, j, k) in [(0, 0, 0), (N, 1, N - 1), (N // 2, N, 1)]:
            l = i + j * N1 + k * N1 * N1
            J8 = 8.0 * _fd_jacobian(jmesh.verts[e], xi[i], xi[j], xi[k])
            ref = lam[e, l] * _sym6(_adj(J8.T @ J8))
            assert np.allclose(G[e, :, l], ref, rtol=0, atol=2e-14 * np.abs(G[e, :, l]).max())


@pytest.mark.parametrize("N", [2, 4])
def test_invariances(N, jmesh):
    """Rotation and translation leave G unchanged; uniform scaling by s scales G by s."""
    xi, w, _ = oracle.gll(N)
    V = jmesh.verts[:4]
    G0, gwj0, _ = oracle.geom_factors(V, N, xi, w)
    Q = meshgen.random_affine(3, max_cond=1.0)  # orthogonal, det +1
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-14)
    V1 = V @ Q.T + np.array([3.0, -1.0, 0.5])
    G1, gwj1, _ = oracle.geom_factors(V1, N, xi, w)
    assert np.allclose(G1, G0, rtol=0, atol=1e-13 * np.abs(G0).max())
    assert np.allclose(gwj1, gwj0, rtol=1e-12, atol=0)
    s = 2.5
    G2, gwj2, _ = oracle.geom_factors(V * s, N, xi, w)
    assert np.allclose(G2, s * G0, rtol=1e-13, atol=1e-16)
    assert np.allclose(gwj2, s**3 * gwj0, rtol=1e-13, atol=0)


@pytest.mark.parametrize("N", [2, 3, 7])
def test_volume_of_unit_cube(N):
    """sum over all nodes of gwj = vol(Omega) = 1 for the jittered unit cube (GLL with N >= 2
    integrates the per-direction quadratic det J exactly)."""
    m = meshgen.jittered_hex(4, 3, 2, alpha=0.15, seed=N)
    xi, w, _ = oracle.gll(N)
    _, gwj, mind = oracle.geom_factors(m.verts, N, xi, w)
    assert mind > 0
    assert gwj.sum() == pytest.approx(1.0, abs=1e-13)


def test_parallelepiped_h():
    mesh, M = meshgen.parallelepiped_hex(2, 3, 4, seed=2)
    h = oracle.parallelepiped_h(mesh.verts)
    J = M @ np.diag(np.array([1 / 2, 1 / 3, 1 / 4]) / 2)
    Ji = np.linalg.inv(J)
    ref = _sym6(np.linalg.det(J) * Ji @ Ji.T)
    assert np.allclose(h, ref[None, :], rtol=1e-13, atol=0)
    xi, w, _ = oracle.gll(3)
    G, _, _ = oracle.geom_factors(mesh.verts, 3, xi, w)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    assert np.allclose(G, h[:, :, None] * W[None, None, :], rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("N", [1, 3])
def test_node_coords(N, jmesh):
    xi, _, _ = oracle.gll(N)
    X = oracle.node_coords(jmesh.verts, N, xi)
    N1 = N + 1
    for e in (0, jmesh.E - 1):
        f = _interp_map(jmesh.verts[e])
        for (i, j, k) in [(0, 0, 0), (N, 0, 0), (0, N, N), (N, N, N), (1, 0, N)]:
            l = i + j * N1 + k * N1 * N1
            assert np.allclose(X[e, :, l], f([xi[i], xi[j], xi[k]])[0], rtol=0, atol=1e-15)
        # corners are the vertices themselves
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    l = a * N + b * N * N1 + c * N * N1 * N1
                    assert np.allclose(X[e, :, l], jmesh.verts[e, a + 2 * b + 4 * c], atol=1e-15)


def test_jacobians_batch_matches_per_node():
    """The all-nodes Jacobian evaluation is the per-node one, node for node (layout check)."""
    m = meshgen.jittered_hex(2, 1, 2, alpha=0.2, seed=9)
    N = 4
    xi, _, _ = oracle.gll(N)
    J = oracle.jacobians(m.verts, N, xi)
    for e in range(m.E):
        for k in range(N + 1):
            for j in range(N + 1):
                for i in range(N + 1):
                    ref = oracle.jacobian(m.verts[e], xi[i], xi[j], xi[k])
                    assert np.array_equal(J[e, i + j * (N + 1) + k * (N + 1) ** 2], ref)
