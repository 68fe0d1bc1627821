"""Pins of the oracle's GLL tables (Table 1) against values the paper prints, closed forms and
independent high-precision / library computations."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
from conftest import golden

NS = list(range(1, 16))


def test_worked_example_n2():
    """Sec. 2.1 prints Xi_2, W_2 and Dhat_2 exactly."""
    g = golden("gll_n2.json")
    xi, w, D = oracle.gll(2)
    assert np.array_equal(xi, np.array(g["xi"]))
    w_ref = np.array([Fraction(n, g["w_den"]) for n in g["w_num"]], dtype=float)
    assert np.allclose(w, w_ref, rtol=0, atol=2e-16)
    assert np.allclose(D, np.array(g["D"]), rtol=0, atol=4e-16)
    # L_2(x) = (3 x^2 - 1) / 2
    c = g["L2_coeffs_x2_x1_x0_times2"]
    for x in (-0.7, 0.1, 0.9):
        L, dL = oracle.legendre(2, x)
        assert L == pytest.approx((c[0] * x * x + c[1] * x + c[2]) / 2, abs=1e-15)
        assert dL == pytest.approx(3 * x, abs=1e-15)


@pytest.mark.parametrize("N", NS)
def test_points_are_gll_roots_numpy(N):
    """Interior points are the roots of L_N' (numpy companion-matrix roots, independent)."""
    xi, _, _ = oracle.gll(N)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    if N > 1:
        roots = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
        assert np.allclose(xi[1:-1], roots, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [3, 5, 7, 9, 11, 15])
def test_points_weights_mpmath(N):
    """50-digit cross-check of points and weights (weights by the Table 1 formula in mpmath)."""
    mpmath.mp.dps = 50
    xi, w, _ = oracle.gll(N)

    def dL(x):
        return mpmath.diff(lambda y: mpmath.legendre(N, y), x)

    for i in range(1, N):
        r = mpmath.findroot(dL, mpmath.mpf(xi[i]))
        assert abs(float(r) - xi[i]) <= 4 * np.spacing(max(abs(xi[i]), 1e-3))
    for i in range(N + 1):
        x = mpmath.mpf(-1) if i == 0 else (mpmath.mpf(1) if i == N else mpmath.findroot(dL, mpmath.mpf(xi[i])))
        wi = 2 / (N * (N + 1) * mpmath.legendre(N, x) ** 2)
        # the recurrence for L_N carries O(N) rounding, doubled by the square
        assert abs(float(wi) - w[i]) <= 4 * N * np.spacing(w[i])


@pytest.mark.parametrize("N", NS)
def test_quadrature_exactness(N):
    """GLL quadrature integrates polynomials of degree <= 2N - 1 exactly; sum w = 2."""
    xi, w, _ = oracle.gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(0, 2 * N):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, xi**p) - exact) < 1e-13, p


@pytest.mark.parametrize("N", NS)
def test_differentiation_exact_on_polynomials(N):
    """Dhat xi^p = p xi^(p-1) for p <= N (D[i][j] = pi_j'(xi_i) differentiates the interpolant)."""
    xi, _, D = oracle.gll(N)
    scale = np.abs(D).sum(axis=1).max()
    for p in range(0, N + 1):
        lhs = D @ xi**p
        rhs = p * xi ** max(p - 1, 0) if p > 0 else np.zeros_like(xi)
        assert np.abs(lhs - rhs).max() < 4e-15 * scale * max(1, p), p


@pytest.mark.parametrize("N", NS)
def test_symmetries(N):
    """Symmetric points/weights; Dhat is centro-antisymmetric; Dhat 1 = 0; the closed-form
    diagonal is -N(N+1)/4, 0, ..., 0, N(N+1)/4."""
    xi, w, D = oracle.gll(N)
    assert np.array_equal(xi, -xi[::-1])
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-16)
    assert np.allclose(D, -D[::-1, ::-1], rtol=0, atol=1e-12 * np.abs(D).max())
    assert np.abs(D.sum(axis=1)).max() < 1e-12
    diag = np.zeros(N + 1)
    diag[0] = -N * (N + 1) / 4.0
    diag[-1] = N * (N + 1) / 4.0
    assert np.allclose(np.diag(D), diag, rtol=0, atol=1e-11)


def test_invalid_order():
    with pytest.raises(ValueError):
        oracle.gll(0)
