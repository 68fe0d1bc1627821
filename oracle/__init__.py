"""CPU oracle for the matrix-free element-local Poisson operator (arXiv 2504.07042).

TEST INFRASTRUCTURE ONLY: the plain double-precision definitions the HIP path is checked
against.  Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  It shares no code with ``paper_2504_07042_amd`` and imports nothing from it.

Thin ctypes wrappers around ``oracle.c`` (numpy in, numpy out).  Each wrapper names the passage
of the paper the C routine evaluates.  ``dense`` holds the brute-force assembled matrices.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(
            os.path.join(_HERE, "oracle.c")):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
    lib.orc_gll.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    lib.orc_gll.restype = ctypes.c_int
    lib.orc_jacobian.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_jacobians.argtypes = [_i64, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_geom_factors.argtypes = [_i64, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_node_coords.argtypes = [_i64, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_parallelepiped_h.argtypes = [_i64, _dp, _dp]
    lib.orc_ax_local.argtypes = [_i64, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp]
    lib.orc_gs_qt.argtypes = [_i64, _i64, _ip, ctypes.c_int, _dp, _dp]
    lib.orc_gs_q.argtypes = [_i64, _i64, _ip, ctypes.c_int, _dp, _dp]
    lib.orc_apply_A.argtypes = [_i64, ctypes.c_int, _dp, _dp, _i64, _ip, _up, _dp, _dp, _dp]
    lib.orc_cg.argtypes = [_i64, ctypes.c_int, _dp, _dp, _i64, _ip, _up, _dp, _dp,
                           ctypes.c_double, ctypes.c_int, _dp]
    lib.orc_cg.restype = ctypes.c_int
    lib.orc_pcg.argtypes = [_i64, ctypes.c_int, _dp, _dp, _i64, _ip, _up, _dp, _dp, _dp,
                            ctypes.c_double, ctypes.c_int, _dp]
    lib.orc_pcg.restype = ctypes.c_int
    lib.orc_ax_diag.argtypes = [_i64, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    _lib = lib
    return lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().orc_set_num_threads(int(n))


def legendre(N: int, x: float):
    """L_N(x), L_N'(x) (Table 1)."""
    L = ctypes.c_double()
    dL = ctypes.c_double()
    _load().orc_legendre(N, float(x), ctypes.byref(L), ctypes.byref(dL))
    return L.value, dL.value


def gll(N: int):
    """GLL points, weights and differentiation matrix D[i][j] = pi_j'(xi_i) (Table 1)."""
    N1 = N + 1
    xi = np.zeros(N1)
    w = np.zeros(N1)
    D = np.zeros((N1, N1))
    if _load().orc_gll(N, _d(xi), _d(w), _d(D)) != 0:
        raise ValueError(f"N={N} unsupported")
    return xi, w, D


def jacobian(V, r: float, s: float, t: float) -> np.ndarray:
    """J[c][d] = d x_c / d r_d of the trilinear map at (r, s, t) (Eq. 5, Eq. 9)."""
    V = _c64(V).reshape(8, 3)
    J = np.zeros((3, 3))
    _load().orc_jacobian(_d(V), float(r), float(s), float(t), _d(J))
    return J


def jacobians(verts, N: int, xi) -> np.ndarray:
    """The Jacobian of Eq. (9) at every GLL node of every element, [E][N1^3][3][3]."""
    verts = _c64(verts)
    E = verts.shape[0]
    J = np.zeros((E, (N + 1) ** 3, 3, 3))
    _load().orc_jacobians(E, N, _d(verts), _d(_c64(xi)), _d(J))
    return J


def geom_factors(verts, N: int, xi, w):
    """(G [E][6][N1^3], gwj [E][N1^3], min det J): Eq. (7) with J from Eq. (9)."""
    verts = _c64(verts)
    E = verts.shape[0]
    Np = (N + 1) ** 3
    G = np.zeros((E, 6, Np))
    gwj = np.zeros((E, Np))
    mind = ctypes.c_double()
    _load().orc_geom_factors(E, N, _d(verts), _d(_c64(xi)), _d(_c64(w)), _d(G), _d(gwj),
                             ctypes.byref(mind))
    return G, gwj, mind.value


def lambda_geo(verts, N: int, xi, w) -> np.ndarray:
    """Per-node scale of the partial recomputation (Sec. 4.2.2; the lambda of Eq. 12):
    lam = 0.125 w_i w_j w_k / det(8J) = w_i w_j w_k / (4096 det J) [E][N1^3], with det J taken
    from the lumped mass gwj = w_i w_j w_k det J of geom_factors (Eq. 7, J from Eq. 9)."""
    _, gwj, _ = geom_factors(verts, N, xi, w)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    return W * W / (4096.0 * gwj)


def ax_local_helmholtz(D, G, gwj, lambda0, lambda1, X) -> np.ndarray:
    """Helmholtz AxLocal (Eq. 3): Y_e = D^T (Lambda0 G_e) D X_e + Lambda1 Gwj X_e, with the nodal
    coefficient fields lambda0, lambda1 [E][N1^3] scaling the factors G [E][6][N1^3] and the
    lumped mass gwj [E][N1^3] node by node (the diagonal matrices of Eq. 3)."""
    lambda0 = np.asarray(lambda0, dtype=np.float64)
    Y = ax_local(D, G * lambda0[:, None, :], X)
    return Y + (np.asarray(lambda1, dtype=np.float64) * gwj)[None] * np.asarray(X, dtype=np.float64).reshape(Y.shape)


def node_coords(verts, N: int, xi) -> np.ndarray:
    """Physical node coordinates [E][3][N1^3] (Eq. 8)."""
    verts = _c64(verts)
    E = verts.shape[0]
    XYZ = np.zeros((E, 3, (N + 1) ** 3))
    _load().orc_node_coords(E, N, _d(verts), _d(_c64(xi)), _d(XYZ))
    return XYZ


def parallelepiped_h(verts) -> np.ndarray:
    """h[E][6] = det J J^-1 J^-T without weights (input of Algorithm 3)."""
    verts = _c64(verts)
    h = np.zeros((verts.shape[0], 6))
    _load().orc_parallelepiped_h(verts.shape[0], _d(verts), _d(h))
    return h


def ax_local(D, G, X) -> np.ndarray:
    """Y = AxLocal(X) = D^T G D X per element (Eq. 3, Poisson; D of Table 1).  G [E][6][N1^3],
    X [nrhs][E][N1^3]."""
    D = _c64(D)
    G = _c64(G)
    X = _c64(X)
    N1 = D.shape[0]
    E = G.shape[0]
    if X.ndim == 2:
        X = X.reshape(1, *X.shape)
    nrhs = X.shape[0]
    assert X.shape == (nrhs, E, N1**3)
    Y = np.zeros_like(X)
    _load().orc_ax_local(E, N1 - 1, _d(D), _d(G), nrhs, _d(X), _d(Y))
    return Y


def ax_envelope(D, G, X) -> np.ndarray:
    """|D|^T |G| |D| |X| (the entrywise error envelope of AxLocal): Eq. 3 evaluated on the
    absolute values."""
    return ax_local(np.abs(D), np.abs(G), np.abs(X))


def gs_qt(l2g, n_global: int, Yl) -> np.ndarray:
    """Q^T: sum local values into global nodes in ascending local order (Eq. 1)."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    Yl = _c64(Yl)
    nrhs = Yl.size // l2g.size
    out = np.zeros((nrhs, n_global))
    _load().orc_gs_qt(l2g.size, n_global, l2g.ctypes.data_as(_ip), nrhs, _d(Yl), _d(out))
    return out


def gs_q(l2g, xg) -> np.ndarray:
    """Q: copy global values to local nodes."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    xg = _c64(xg)
    n_global = xg.shape[-1]
    nrhs = xg.size // n_global
    out = np.zeros((nrhs, l2g.size))
    _load().orc_gs_q(l2g.size, n_global, l2g.ctypes.data_as(_ip), nrhs, _d(xg), _d(out))
    return out


def apply_A(N, D, G, l2g, n_global, mask, x) -> np.ndarray:
    """y = mask o Q^T AxLocal(Q x) (Eq. 1, Dirichlet rows zeroed)."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    x = _c64(x)
    y = np.zeros(n_global)
    work = np.zeros(2 * l2g.size)
    mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).ctypes.data_as(_up)
    _load().orc_apply_A(G.shape[0], N, _d(_c64(D)), _d(_c64(G)), n_global, l2g.ctypes.data_as(_ip),
                        mp, _d(x), _d(y), _d(work))
    return y


def cg(N, D, G, l2g, n_global, mask, b, x0=None, rtol=1e-10, max_it=10000):
    """Plain CG on the assembled operator.  Returns (x, iterations, true relative residual)."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    b = _c64(b)
    x = np.zeros(n_global) if x0 is None else _c64(x0).copy()
    rel = ctypes.c_double()
    mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).ctypes.data_as(_up)
    it = _load().orc_cg(G.shape[0], N, _d(_c64(D)), _d(_c64(G)), n_global, l2g.ctypes.data_as(_ip),
                        mp, _d(b), _d(x), float(rtol), int(max_it), ctypes.byref(rel))
    return x, it, rel.value


def ax_diag(D, G) -> np.ndarray:
    """Diagonal of every element matrix D^T G_e D of Eq. (3) (Poisson), [E][N1^3]."""
    D = _c64(D)
    G = _c64(G)
    N1 = D.shape[0]
    out = np.zeros((G.shape[0], N1**3))
    _load().orc_ax_diag(G.shape[0], N1 - 1, _d(D), _d(G), _d(out))
    return out


def jacobi_dinv(D, G, l2g, n_global, mask) -> np.ndarray:
    """Inverse diagonal of the assembled operator (Q^T of the element diagonals, Eq. 1), zero on
    the Dirichlet nodes (their rows of the assembled operator are zero)."""
    dg = gs_qt(l2g, n_global, ax_diag(D, G).reshape(1, -1))[0]
    m = np.zeros(n_global, dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    out = np.zeros(n_global)
    out[~m] = 1.0 / dg[~m]
    return out


def pcg(N, D, G, l2g, n_global, mask, b, dinv, x0=None, rtol=1e-10, max_it=10000):
    """Jacobi-preconditioned CG (M^-1 = diag(dinv)).  Returns (x, iterations, true rel. residual)."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    b = _c64(b)
    x = np.zeros(n_global) if x0 is None else _c64(x0).copy()
    rel = ctypes.c_double()
    mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).ctypes.data_as(_up)
    it = _load().orc_pcg(G.shape[0], N, _d(_c64(D)), _d(_c64(G)), n_global, l2g.ctypes.data_as(_ip), mp,
                         _d(b), _d(_c64(dinv)), _d(x), float(rtol), int(max_it), ctypes.byref(rel))
    return x, it, rel.value


def poisson_rhs(N, verts, xi, w, l2g, n_global, mask):
    """Right-hand side of -Lap u = f for u = sin(pi x) sin(pi y) sin(pi z):
    f = 3 pi^2 u at the physical nodes, b = mask o Q^T (gwj o f) (GLL-lumped mass, Eq. 7)."""
    XYZ = node_coords(verts, N, xi)
    _, gwj, _ = geom_factors(verts, N, xi, w)
    u = np.sin(np.pi * XYZ[:, 0]) * np.sin(np.pi * XYZ[:, 1]) * np.sin(np.pi * XYZ[:, 2])
    f = 3.0 * np.pi**2 * u
    b = gs_qt(l2g, n_global, (gwj * f).reshape(1, -1))[0]
    b[np.asarray(mask, dtype=bool)] = 0.0
    return b, u
