"""Brute-force dense matrices for tiny cases (TEST INFRASTRUCTURE ONLY).

The discrete gradient D = [I x I x Dhat; I x Dhat x I; Dhat x I x I] of Table 1 is formed as
explicit Kronecker products, and the element matrix of Eq. (3) (Poisson: Lambda0 = I,
Lambda1 = 0) as D^T [G00 G01 G02; G01 G11 G12; G02 G12 G22] D with diagonal blocks.  No sum
factorisation is used here, so this is an independent route to the operator that
``oracle.ax_local`` evaluates by Algorithm 1.
"""
from __future__ import annotations

import numpy as np


def gradient(Dhat: np.ndarray) -> np.ndarray:
    """The 3 N1^3 x N1^3 discrete gradient of Table 1 (node index i + j N1 + k N1^2, so the
    fastest index i is the rightmost Kronecker factor)."""
    N1 = Dhat.shape[0]
    I = np.eye(N1)
    Dr = np.kron(I, np.kron(I, Dhat))
    Ds = np.kron(I, np.kron(Dhat, I))
    Dt = np.kron(Dhat, np.kron(I, I))
    return np.vstack([Dr, Ds, Dt])


def element_matrix(Dhat: np.ndarray, G_e: np.ndarray) -> np.ndarray:
    """A^(e) = D^T Gblock D (Eq. 3, Poisson), G_e [6][N1^3] in order 00,01,02,11,12,22."""
    Dg = gradient(Dhat)
    g = G_e
    blocks = [[g[0], g[1], g[2]], [g[1], g[3], g[4]], [g[2], g[4], g[5]]]
    Gb = np.block([[np.diag(b) for b in row] for row in blocks])
    return Dg.T @ Gb @ Dg


def assembled_matrix(Dhat, G, l2g, n_global, mask=None) -> np.ndarray:
    """A = Q^T blockdiag(A^(e)) Q (Eq. 1), with Dirichlet rows and columns replaced by zero."""
    N1 = Dhat.shape[0]
    Np = N1**3
    E = G.shape[0]
    A = np.zeros((n_global, n_global))
    for e in range(E):
        Ae = element_matrix(Dhat, G[e])
        idx = np.asarray(l2g[e * Np:(e + 1) * Np])
        A[np.ix_(idx, idx)] += Ae
    if mask is not None:
        m = np.asarray(mask, dtype=bool)
        A[m, :] = 0.0
        A[:, m] = 0.0
    return A
