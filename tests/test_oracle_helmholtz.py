"""Pins of the oracle's Helmholtz AxLocal (Eq. 2-3: coefficient fields lambda0 on the stiffness,
lambda1 on the lumped mass) against closed-form energies on the unit cube and the Poisson
special case."""
import numpy as np
import pytest

import oracle
from paper_2504_07042_amd import meshgen


def _setup(N, nx=2, ny=2, nz=2, alpha=0.15, seed=5):
    m = meshgen.jittered_hex(nx, ny, nz, alpha=alpha, seed=seed)
    xi, w, D = oracle.gll(N)
    G, gwj, _ = oracle.geom_factors(m.verts, N, xi, w)
    return m, xi, w, D, G, gwj


@pytest.mark.parametrize("N", [1, 3])
def test_poisson_special_case(N):
    m, xi, w, D, G, gwj = _setup(N)
    X = meshgen.random_nodal(m.E, N, nrhs=2, seed=2)
    one, zero = np.ones_like(gwj), np.zeros_like(gwj)
    assert np.array_equal(oracle.ax_local_helmholtz(D, G, gwj, one, zero, X), oracle.ax_local(D, G, X))


@pytest.mark.parametrize("N", [2, 4])
def test_constant_field_mass(N):
    """u = 1: the stiffness part vanishes (D 1 = 0) and the sum of all entries of Y is
    lambda1 vol(Omega) = lambda1 for the unit cube, whatever lambda0 is."""
    m, xi, w, D, G, gwj = _setup(N)
    rng = np.random.default_rng(4)
    lam0 = rng.uniform(0.5, 2.0, gwj.shape)
    c = 2.75
    Y = oracle.ax_local_helmholtz(D, G, gwj, lam0, np.full_like(gwj, c), np.ones((1, *gwj.shape)))
    assert float(Y.sum()) == pytest.approx(c, rel=1e-12)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_linear_field_energy_on_boxes(N):
    """u = x on an undistorted 2x2x2 box mesh of the unit cube with lambda0 = x and lambda1 = c:
    u^T A u = int x |grad x|^2 + c int x^2 = 1/2 + c/3 (GLL with N >= 2 integrates both exactly)."""
    m, xi, w, D, G, gwj = _setup(N, alpha=0.0)
    XYZ = oracle.node_coords(m.verts, N, xi)
    x = XYZ[:, 0, :]
    c = 1.5
    Y = oracle.ax_local_helmholtz(D, G, gwj, x, np.full_like(gwj, c), x[None])
    assert float(np.sum(x[None] * Y)) == pytest.approx(0.5 + c / 3.0, rel=1e-12)
