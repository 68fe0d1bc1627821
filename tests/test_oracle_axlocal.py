"""Pins of the oracle's AxLocal (Algorithm 1, Poisson) against brute-force dense element
matrices (Eq. 3), the textbook tensor-product form on a box, and invariants of the operator."""
import numpy as np
import pytest

import oracle
from oracle import dense
from conftest import golden
from paper_2504_07042_amd import meshgen


def _setup(N, nx=2, ny=2, nz=1, alpha=0.15, seed=3):
    m = meshgen.jittered_hex(nx, ny, nz, alpha=alpha, seed=seed)
    xi, w, D = oracle.gll(N)
    G, gwj, mind = oracle.geom_factors(m.verts, N, xi, w)
    assert mind > 0
    return m, xi, w, D, G, gwj


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_loops_match_dense(N):
    m, xi, w, D, G, _ = _setup(N)
    X = meshgen.random_nodal(m.E, N, nrhs=2, seed=1)
    Y = oracle.ax_local(D, G, X)
    for e in range(m.E):
        Ae = dense.element_matrix(D, G[e])
        for c in range(2):
            ref = Ae @ X[c, e]
            assert np.linalg.norm(Y[c, e] - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_symmetric_psd_constant_nullspace(N):
    m, xi, w, D, G, _ = _setup(N, 1, 1, 1)
    Ae = dense.element_matrix(D, G[0])
    assert np.abs(Ae - Ae.T).max() <= 1e-14 * np.abs(Ae).max()
    ev = np.linalg.eigvalsh(0.5 * (Ae + Ae.T))
    assert ev.min() >= -1e-13 * ev.max()
    one = np.ones((1, 1, (N + 1) ** 3))
    Y = oracle.ax_local(D, G, one)
    assert np.abs(Y).max() <= 1e-13 * np.abs(G).max() * np.abs(D).sum(axis=1).max() ** 2


@pytest.mark.parametrize("N", [2, 3, 6])
def test_patch_energy_linear_field(N):
    """For u = a . x (linear in physical space), u^T A u = |a|^2 vol(Omega) exactly (the energy
    integral of a constant gradient); holds on trilinear elements for N >= 2."""
    m, xi, w, D, G, gwj = _setup(N, 2, 2, 2)
    XYZ = oracle.node_coords(m.verts, N, xi)
    a = np.array([0.3, -1.2, 0.7])
    u = np.einsum("c,ecl->el", a, XYZ)[None]
    Y = oracle.ax_local(D, G, u)
    energy = float(np.sum(u * Y))
    vol = gwj.sum()
    assert vol == pytest.approx(1.0, abs=1e-13)
    assert energy == pytest.approx(np.dot(a, a) * vol, rel=1e-12)
    # element by element too
    for e in range(m.E):
        assert np.sum(u[0, e] * Y[0, e]) == pytest.approx(np.dot(a, a) * gwj[e].sum(), rel=1e-11)


def test_box_tensor_form_and_1d_stiffness():
    """On an undeformed cube of side h, A^(e) = h/2 (Ahat x M x M + M x Ahat x M + M x M x Ahat)
    with M = diag(W) and Ahat = Dhat^T M Dhat; for N = 2 Ahat is the exact quadratic stiffness."""
    g = golden("stiffness_1d_n2.json")
    xi, w, D = oracle.gll(2)
    Ahat = D.T @ np.diag(w) @ D
    assert np.allclose(Ahat, np.array(g["A_times_6"]) / g["scale_den"], rtol=0, atol=2e-15)
    for N in (2, 4):
        xi, w, D = oracle.gll(N)
        hside = 0.37
        V = meshgen.box_element(hside, hside, hside)
        G, _, _ = oracle.geom_factors(V, N, xi, w)
        M = np.diag(w)
        Ah = D.T @ M @ D
        ref = hside / 2 * (np.kron(Ah, np.kron(M, M)) + np.kron(M, np.kron(Ah, M)) + np.kron(M, np.kron(M, Ah)))
        Ae = dense.element_matrix(D, G[0])
        assert np.abs(Ae - ref).max() <= 1e-14 * np.abs(ref).max()
        X = meshgen.random_nodal(1, N, seed=4)
        Y = oracle.ax_local(D, G, X)
        assert np.allclose(Y[0, 0], ref @ X[0, 0], rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("N", [2, 3])
def test_assembled_patch_interior_zero(N):
    """After assembly, (A u_lin) vanishes at interior global nodes (consistency of the
    discretisation for linear fields on trilinear meshes)."""
    m, xi, w, D, G, gwj = _setup(N, 3, 3, 3)
    l2g, ng, mask = meshgen.global_numbering(3, 3, 3, N)
    XYZ = oracle.node_coords(m.verts, N, xi)
    a = np.array([1.0, 2.0, -0.5])
    ul = np.einsum("c,ecl->el", a, XYZ).reshape(-1)
    ug = np.zeros(ng)
    ug[l2g] = ul
    y = oracle.apply_A(N, D, G, l2g, ng, None, ug)
    interior = mask == 0
    scale = np.abs(oracle.gs_qt(l2g, ng, oracle.ax_envelope(D, G, ul.reshape(1, m.E, -1)))).max()
    assert np.abs(y[interior]).max() <= 1e-12 * scale


def test_envelope_bounds_output():
    m, xi, w, D, G, _ = _setup(3)
    X = meshgen.random_nodal(m.E, 3, seed=9)
    Y = oracle.ax_local(D, G, X)
    env = oracle.ax_envelope(D, G, X)
    assert np.all(np.abs(Y) <= env * (1 + 1e-12))
