"""MI355X (gfx950) matrix-free element-local Poisson operator with on-the-fly geometric factors
(after arXiv 2504.07042).

A thin ctypes binding of ``libaxhosfem.so`` (C ABI in ``include/axhosfem.h``).  PyTorch supplies
device memory and the current HIP stream; every step of the operator runs in the library's HIP
kernels.  Nothing here falls back to the CPU: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import meshgen  # noqa: F401  (seeded synthetic inputs)

PKG = os.path.dirname(os.path.abspath(__file__))
# AXHOSFEM_LIB selects another build of the same library (e.g. the LDS-poisoned debug twin)
LIBPATH = os.environ.get("AXHOSFEM_LIB") or os.path.join(PKG, "libaxhosfem.so")

AX_OK, AX_ERR_ARG, AX_ERR_UNSUPPORTED, AX_ERR_HIP, AX_ERR_NOMEM, AX_ERR_NOT_CONVERGED, AX_ERR_BREAKDOWN = (
    0, -1, -2, -3, -4, -5, -6)
AX_TRILINEAR, AX_PARALLELEPIPED, AX_STORED_G = 0, 1, 2
AX_FP64, AX_FP32, AX_FP16_ACC32 = 0, 1, 2
AX_REFINE_RESTART, AX_REFINE_RELIABLE = 0, 1
AX_PRECOND_NONE, AX_PRECOND_JACOBI = 0, 1
AX_PROBE_FMA_F64, AX_PROBE_FMA_F32, AX_PROBE_MFMA_F64, AX_PROBE_MFMA_F32, AX_PROBE_MIX_F64 = 0, 1, 2, 3, 4
(AX_TUNE_TRILINEAR, AX_TUNE_PARALLELEPIPED, AX_TUNE_STORED, AX_TUNE_PARTIAL, AX_TUNE_HELMHOLTZ,
 AX_TUNE_BATCHED) = 0, 1, 2, 3, 4, 5
AX_KERNEL_AUTO, AX_KERNEL_TILE, AX_KERNEL_ITEM = 0, 1, 2
GS_QT, GS_Q, GS_QQT = 0, 1, 2

_STATUS = {0: "AX_OK", -1: "AX_ERR_ARG", -2: "AX_ERR_UNSUPPORTED", -3: "AX_ERR_HIP",
           -4: "AX_ERR_NOMEM", -5: "AX_ERR_NOT_CONVERGED", -6: "AX_ERR_BREAKDOWN"}


class AxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)


class AxProblem(ctypes.Structure):
    _fields_ = [("E", _i64), ("N", _int), ("geom", _int), ("geo", _vp), ("D", _vp), ("xi", _vp),
                ("w", _vp), ("n_global", _i64), ("l2g", _vp), ("gptr", _vp), ("gidx", _vp),
                ("mask", _vp)]


class AxCgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_it", _int), ("inner_prec", _int),
                ("inner_rtol", ctypes.c_double), ("max_outer", _int), ("workspace", _vp),
                ("workspace_bytes", ctypes.c_size_t), ("use_graph", _int), ("refine", _int), ("precond", _int)]


class AxBatchPlan(ctypes.Structure):
    _fields_ = [("n_items", _i64), ("nrhs", _int), ("prec", _int), ("bytes", ctypes.c_size_t),
                ("n_mesh", _int), ("gather", _int), ("order_first", _i64 * 11), ("order_count", _i64 * 11),
                ("order_variant", _int * 11)]


class AxTune(ctypes.Structure):
    _fields_ = [("kernel", _int), ("tile_alt", _int), ("item_alt", _int), ("waves_alt", _int),
                ("grid_mult", _int), ("kernel_used", _int), ("elems_per_group", _int), ("block", _int),
                ("waves", _int)]


class AxCgReport(ctypes.Structure):
    _fields_ = [("status", _int), ("outer_it", _int), ("inner_it_total", _int),
                ("rel_res_true", ctypes.c_double), ("seconds", ctypes.c_double)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "ax_last_error": (ctypes.c_char_p, []),
    "ax_version": (ctypes.c_char_p, []),
    "ax_gll": (_int, [_int, _vp, _vp, _vp]),
    "ax_tune_set": (_int, [_int, _int, _int, ctypes.POINTER(AxTune)]),
    "ax_tune_get": (_int, [_int, _int, _int, ctypes.POINTER(AxTune)]),
    "ax_local": (_int, [_i64, _int, _int, _vp, _vp, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "ax_local_precomputedG": (_int, [_i64, _int, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "ax_local_vector": (_int, [_i64, _int, _int, _vp, _vp, _vp, _vp, _int, _vp, _vp, _vp]),
    "ax_local_gathered": (_int, [_i64, _int, _int, _vp, _vp, _vp, _vp, _int, _int, _vp, _i64, _vp, _vp, _vp]),
    "ax_local_gathered_energy": (_int, [_i64, _int, _int, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "ax_geom_factors": (_int, [_i64, _int, _vp, _vp, _vp, _int, _vp, _vp, _vp]),
    "ax_local_partial": (_int, [_i64, _int, _vp, _vp, _vp, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "ax_geom_lambda": (_int, [_i64, _int, _vp, _vp, _vp, _int, _vp, _vp]),
    "ax_local_helmholtz": (_int, [_i64, _int, _vp, _vp, _vp, _vp, _vp, _int, _int, _vp, _vp, _vp]),
    "ax_helmholtz_factors": (_int, [_i64, _int, _vp, _vp, _vp, _vp, _vp, _int, _vp, _vp]),
    "ax_parallelepiped_factors": (_int, [_i64, _vp, _vp, _vp]),
    "ax_local_diag": (_int, [_i64, _int, _int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ax_node_coords": (_int, [_i64, _int, _vp, _vp, _vp, _vp]),
    "ax_check_mesh": (_int, [_i64, _int, _vp, _vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double), _vp]),
    "gs_build_csr": (_int, [_i64, _i64, _vp, _vp, _vp]),
    "gs_assemble": (_int, [_i64, _i64, _vp, _vp, _vp, _vp, _int, _int, _int, _vp, _vp, _vp]),
    "cg_workspace_bytes": (_int, [ctypes.POINTER(AxProblem), _int, ctypes.POINTER(AxCgOpts),
                                  ctypes.POINTER(ctypes.c_size_t)]),
    "cg_solve": (_int, [ctypes.POINTER(AxProblem), _int, _vp, _vp, ctypes.POINTER(AxCgOpts),
                        ctypes.POINTER(AxCgReport), _vp]),
    "ax_batched_workspace_bytes": (_int, [_int, ctypes.POINTER(AxProblem),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "ax_batched_prepare": (_int, [_int, ctypes.POINTER(AxProblem), _int, _int, _vp, _vp, _vp, _vp,
                                  ctypes.c_size_t, ctypes.c_void_p]),
    "ax_local_batched": (_int, [ctypes.c_void_p, _vp, _vp]),
    "ax_probe_copy": (_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "ax_probe_compute_elems": (_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "ax_probe_compute": (_int, [_int, _int, _vp, ctypes.POINTER(ctypes.c_double), _vp]),
    "ax_local_batched_noalloc": (_int, [_int, ctypes.POINTER(AxProblem), _int, _int, _vp, _vp, _vp, _vp]),
    "cg_batched_workspace_bytes": (_int, [_int, ctypes.POINTER(AxProblem), _i64, _int, ctypes.POINTER(AxCgOpts),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "cg_solve_batched": (_int, [_int, ctypes.POINTER(AxProblem), _i64, _vp, _vp, _vp, _vp, _int, _vp, _vp,
                                ctypes.POINTER(AxCgOpts), ctypes.POINTER(AxCgReport), _vp]),
}


def lib():
    """Load libaxhosfem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        # launch shapes picked by the autotuner for this architecture, if a cache exists
        from . import autotune
        autotune.load()
    return _lib


def _check(code: int):
    if code != AX_OK:
        raise AxError(code, lib().ax_last_error().decode())
    return code


def _np_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def gll(N: int):
    """GLL points, weights and differentiation matrix from the library (Table 1)."""
    N1 = N + 1
    xi = np.zeros(N1)
    w = np.zeros(N1)
    D = np.zeros((N1, N1))
    _check(lib().ax_gll(N, _np_ptr(xi), _np_ptr(w), _np_ptr(D)))
    return xi, w, D


class Basis:
    """Host copies of the GLL tables of order N (passed to every kernel call)."""

    def __init__(self, N: int):
        self.N = N
        self.xi, self.w, self.D = gll(N)
        self.xi = np.ascontiguousarray(self.xi)
        self.w = np.ascontiguousarray(self.w)
        self.D = np.ascontiguousarray(self.D)


def _nrhs(X, E, N):
    NP = (N + 1) ** 3
    if X.dim() == 3:
        assert X.shape[1] == E and X.shape[2] == NP, "X must be [nrhs][E][N1^3]"
        return X.shape[0]
    assert X.numel() == E * NP, "X must be [E][N1^3] or [nrhs][E][N1^3]"
    return 1


def _prec_dtype(prec):
    import torch
    return torch.float64 if prec == AX_FP64 else torch.float32


def ax_local(X, geo, basis: Basis, geom=AX_TRILINEAR, prec=AX_FP64, out=None, stream=None):
    """Y = AxLocal(X) with on-the-fly factors.  X [nrhs][E][N1^3] (or [E][N1^3]) device tensor;
    geo: vertices [E][8][3] (trilinear) or h [E][6] (parallelepiped), float64 device."""
    import torch
    E = geo.shape[0]
    nrhs = _nrhs(X, E, basis.N)
    assert X.dtype == _prec_dtype(prec) and geo.dtype == torch.float64
    Y = torch.empty_like(X) if out is None else out
    _check(lib().ax_local(E, basis.N, geom, _dptr(geo), _np_ptr(basis.D), _np_ptr(basis.xi),
                          _np_ptr(basis.w), nrhs, prec, _dptr(X), _dptr(Y), _stream(stream)))
    return Y


def ax_local_vector(X, geo, basis: Basis, geom=AX_TRILINEAR, prec=AX_FP64, out=None, stream=None):
    """Y = AxLocal(X) for a vector field: X [E][3][N1^3] device tensor (the three components of an
    element contiguous); the element's geometric set-up serves all three (Sec. 4.1)."""
    import torch
    E = geo.shape[0]
    assert X.dim() == 3 and X.shape[0] == E and X.shape[1] == 3 and X.shape[2] == (basis.N + 1) ** 3
    assert X.dtype == _prec_dtype(prec) and geo.dtype == torch.float64
    Y = torch.empty_like(X) if out is None else out
    _check(lib().ax_local_vector(E, basis.N, geom, _dptr(geo), _np_ptr(basis.D), _np_ptr(basis.xi),
                                 _np_ptr(basis.w), prec, _dptr(X), _dptr(Y), _stream(stream)))
    return Y


def ax_local_gathered(Xg, l2g, geo, basis: Basis, geom=AX_TRILINEAR, prec=AX_FP64, out=None, stream=None):
    """Y = AxLocal(Q Xg) with the gather fused into the load: Xg [nrhs][n_global] (or [n_global])
    global device tensor, l2g int32 device tensor [E*N1^3]; returns Y [nrhs][E][N1^3]."""
    import torch
    E = geo.shape[0]
    NP = (basis.N + 1) ** 3
    ng = Xg.shape[-1]
    nrhs = Xg.shape[0] if Xg.dim() == 2 else 1
    assert Xg.dtype == _prec_dtype(prec) and l2g.dtype == torch.int32 and l2g.numel() == E * NP
    Y = torch.empty((nrhs, E, NP), dtype=Xg.dtype, device=Xg.device) if out is None else out
    _check(lib().ax_local_gathered(E, basis.N, geom, _dptr(geo), _np_ptr(basis.D), _np_ptr(basis.xi),
                                   _np_ptr(basis.w), nrhs, prec, _dptr(l2g), ng, _dptr(Xg), _dptr(Y),
                                   _stream(stream)))
    return Y


def ax_local_gathered_energy(Xg, l2g, geo, basis: Basis, geom=AX_TRILINEAR, stream=None):
    """FP32 Y = AxLocal(Q Xg) for one column plus its energy sum_e X_e^T Y_e (a one-element FP64
    device tensor); Xg [n_global] float32 device tensor.  Returns (Y [E][N1^3], energy)."""
    import torch
    E = geo.shape[0]
    NP = (basis.N + 1) ** 3
    assert Xg.dtype == torch.float32 and Xg.dim() == 1 and l2g.dtype == torch.int32 and l2g.numel() == E * NP
    Y = torch.empty((E, NP), dtype=torch.float32, device=Xg.device)
    work = torch.empty(max(E, 1), dtype=torch.float64, device=Xg.device)
    energy = torch.empty(1, dtype=torch.float64, device=Xg.device)
    _check(lib().ax_local_gathered_energy(E, basis.N, geom, _dptr(geo), _np_ptr(basis.D), _np_ptr(basis.xi),
                                          _np_ptr(basis.w), _dptr(l2g), Xg.shape[0], _dptr(Xg), _dptr(Y),
                                          _dptr(work), _dptr(energy), _stream(stream)))
    return Y, energy


def ax_local_precomputedG(X, G, basis: Basis, prec=AX_FP64, out=None, stream=None):
    """Y = AxLocal(X) with the six factors read from G [E][6][N1^3]."""
    import torch
    E = G.shape[0]
    nrhs = _nrhs(X, E, basis.N)
    assert X.dtype == _prec_dtype(prec) and G.dtype == _prec_dtype(prec)
    Y = torch.empty_like(X) if out is None else out
    _check(lib().ax_local_precomputedG(E, basis.N, _dptr(G), _np_ptr(basis.D), nrhs, prec,
                                       _dptr(X), _dptr(Y), _stream(stream)))
    return Y


def ax_local_partial(X, verts, lam, basis: Basis, prec=AX_FP64, out=None, stream=None):
    """Y = AxLocal(X) on trilinear elements with partial recomputation: the per-node scale lam
    [E][N1^3] (from geom_lambda) is read, K and adj(K) are recomputed (Sec. 4.2.2)."""
    import torch
    E = verts.shape[0]
    nrhs = _nrhs(X, E, basis.N)
    assert X.dtype == _prec_dtype(prec) and lam.dtype == _prec_dtype(prec) and verts.dtype == torch.float64
    Y = torch.empty_like(X) if out is None else out
    _check(lib().ax_local_partial(E, basis.N, _dptr(verts), _dptr(lam), _np_ptr(basis.D), _np_ptr(basis.xi),
                                  _np_ptr(basis.w), nrhs, prec, _dptr(X), _dptr(Y), _stream(stream)))
    return Y


def ax_local_helmholtz(X, verts, L23, basis: Basis, prec=AX_FP64, out=None, stream=None):
    """Y = Helmholtz AxLocal(X) (Eq. 3) on trilinear elements with the merged scalar factors L23
    [E][2][N1^3] from helmholtz_factors (Sec. 4.2.1)."""
    import torch
    E = verts.shape[0]
    nrhs = _nrhs(X, E, basis.N)
    assert X.dtype == _prec_dtype(prec) and L23.dtype == _prec_dtype(prec) and verts.dtype == torch.float64
    Y = torch.empty_like(X) if out is None else out
    _check(lib().ax_local_helmholtz(E, basis.N, _dptr(verts), _dptr(L23), _np_ptr(basis.D), _np_ptr(basis.xi),
                                    _np_ptr(basis.w), nrhs, prec, _dptr(X), _dptr(Y), _stream(stream)))
    return Y


def helmholtz_factors(verts, lambda0, lambda1, basis: Basis, prec=AX_FP64, stream=None):
    """Merged scalar factors L23 [E][2][N1^3]: lam * lambda0 and gwj * lambda1 per node, from the
    nodal coefficient fields lambda0, lambda1 (float64 [E][N1^3] device tensors)."""
    import torch
    E = verts.shape[0]
    NP = (basis.N + 1) ** 3
    assert lambda0.shape == (E, NP) and lambda1.shape == (E, NP)
    assert lambda0.dtype == torch.float64 and lambda1.dtype == torch.float64
    L23 = torch.empty((E, 2, NP), dtype=_prec_dtype(prec), device=verts.device)
    _check(lib().ax_helmholtz_factors(E, basis.N, _dptr(verts), _np_ptr(basis.xi), _np_ptr(basis.w),
                                      _dptr(lambda0), _dptr(lambda1), prec, _dptr(L23), _stream(stream)))
    return L23


def geom_lambda(verts, basis: Basis, prec=AX_FP64, stream=None):
    """Per-node scale lam [E][N1^3] = 0.125 w_i w_j w_k / det(8J) for ax_local_partial."""
    import torch
    E = verts.shape[0]
    lam = torch.empty((E, (basis.N + 1) ** 3), dtype=_prec_dtype(prec), device=verts.device)
    _check(lib().ax_geom_lambda(E, basis.N, _dptr(verts), _np_ptr(basis.xi), _np_ptr(basis.w), prec,
                                _dptr(lam), _stream(stream)))
    return lam


def geom_factors(verts, basis: Basis, prec=AX_FP64, want_G=True, want_gwj=False, stream=None):
    """Stored factors G [E][6][N1^3] (Eq. 7) and/or the lumped mass gwj [E][N1^3] (FP64)."""
    import torch
    E = verts.shape[0]
    NP = (basis.N + 1) ** 3
    G = torch.empty((E, 6, NP), dtype=_prec_dtype(prec), device=verts.device) if want_G else None
    gwj = torch.empty((E, NP), dtype=torch.float64, device=verts.device) if want_gwj else None
    _check(lib().ax_geom_factors(E, basis.N, _dptr(verts), _np_ptr(basis.xi), _np_ptr(basis.w), prec,
                                 _dptr(G) if G is not None else None,
                                 _dptr(gwj) if gwj is not None else None, _stream(stream)))
    return G, gwj


def local_diag(geo, basis: Basis, geom=AX_TRILINEAR, stream=None):
    """Diagonal of every element matrix D^T G_e D (Eq. 3), factors recomputed: [E][N1^3] FP64."""
    import torch
    E = geo.shape[0]
    out = torch.empty((E, (basis.N + 1) ** 3), dtype=torch.float64, device=geo.device)
    _check(lib().ax_local_diag(E, basis.N, geom, _dptr(geo), _np_ptr(basis.D), _np_ptr(basis.xi),
                               _np_ptr(basis.w), _dptr(out), _stream(stream)))
    return out


def check_mesh(verts, basis: Basis, stream=None):
    """det J > 0 at every GLL node of every element (Eq. 8-9)?  Returns (bad_element, min_det):
    bad_element is -1 for a valid mesh, else the lowest element with det J <= 0 (or not finite)
    at a node; min_det is the smallest finite det J.  Other errors raise AxError."""
    bad = _i64(-1)
    dmin = ctypes.c_double(0.0)
    code = lib().ax_check_mesh(verts.shape[0], basis.N, _dptr(verts), _np_ptr(basis.xi), ctypes.byref(bad),
                               ctypes.byref(dmin), _stream(stream))
    if code not in (AX_OK, AX_ERR_ARG) or (code == AX_ERR_ARG and bad.value < 0):
        _check(code)
    return bad.value, dmin.value


def parallelepiped_factors(verts, stream=None):
    import torch
    h = torch.empty((verts.shape[0], 6), dtype=torch.float64, device=verts.device)
    _check(lib().ax_parallelepiped_factors(verts.shape[0], _dptr(verts), _dptr(h), _stream(stream)))
    return h


def node_coords(verts, basis: Basis, stream=None):
    import torch
    E = verts.shape[0]
    XYZ = torch.empty((E, 3, (basis.N + 1) ** 3), dtype=torch.float64, device=verts.device)
    _check(lib().ax_node_coords(E, basis.N, _dptr(verts), _np_ptr(basis.xi), _dptr(XYZ), _stream(stream)))
    return XYZ


def gs_build_csr(l2g: np.ndarray, n_global: int):
    """Host CSR inverse of l2g (ascending local ids)."""
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    gptr = np.zeros(n_global + 1, dtype=np.int64)
    gidx = np.zeros(l2g.size, dtype=np.int32)
    _check(lib().gs_build_csr(l2g.size, n_global, _np_ptr(l2g), _np_ptr(gptr), _np_ptr(gidx)))
    return gptr, gidx


class GatherScatter:
    """Device copies of l2g, its CSR inverse and the Dirichlet mask of one mesh."""

    def __init__(self, l2g: np.ndarray, n_global: int, mask=None, device="cuda"):
        import torch
        gptr, gidx = gs_build_csr(l2g, n_global)
        self.n_local = int(l2g.size)
        self.n_global = int(n_global)
        self.l2g = torch.from_numpy(np.ascontiguousarray(l2g, dtype=np.int32)).to(device)
        self.gptr = torch.from_numpy(gptr).to(device)
        self.gidx = torch.from_numpy(gidx).to(device)
        self.mask = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(device)

    def apply(self, x, mode, out=None, use_mask=True, stream=None):
        import torch
        dtype = AX_FP64 if x.dtype == torch.float64 else AX_FP32
        n_in = self.n_local if mode in (GS_QT, GS_QQT) else self.n_global
        nrhs = x.numel() // n_in
        n_out = self.n_global if mode == GS_QT else self.n_local
        if out is None:
            out = torch.empty((nrhs, n_out), dtype=x.dtype, device=x.device)
        m = self.mask if use_mask else None
        _check(lib().gs_assemble(self.n_local, self.n_global, _dptr(self.l2g), _dptr(self.gptr),
                                 _dptr(self.gidx), _dptr(m) if m is not None else None, mode, nrhs,
                                 dtype, _dptr(x), _dptr(out), _stream(stream)))
        return out


class Problem:
    """A Poisson problem on one mesh held on the device: geometry, GLL tables and the
    gather-scatter maps (the ax_problem of the C ABI)."""

    def __init__(self, geo, basis: Basis, gs: GatherScatter, geom=AX_TRILINEAR):
        self.geo = geo
        self.basis = basis
        self.gs = gs
        self.geom = geom
        self.E = geo.shape[0]

    def c_struct(self) -> AxProblem:
        b = self.basis
        gs = self.gs
        return AxProblem(self.E, b.N, self.geom, self.geo.data_ptr(), b.D.ctypes.data, b.xi.ctypes.data,
                         b.w.ctypes.data, gs.n_global, gs.l2g.data_ptr(), gs.gptr.data_ptr(),
                         gs.gidx.data_ptr(), gs.mask.data_ptr() if gs.mask is not None else None)

    def apply(self, x, prec=AX_FP64, stream=None):
        """y = mask o Q^T AxLocal(Q x) on global vectors [nrhs][n_global]."""
        import torch
        xl = self.gs.apply(x, GS_Q, stream=stream)
        xl = xl.view(xl.shape[0], self.E, -1)
        if self.geom == AX_TRILINEAR:
            yl = ax_local(xl, self.geo, self.basis, AX_TRILINEAR, prec, stream=stream)
        else:
            yl = ax_local(xl, self.geo, self.basis, AX_PARALLELEPIPED, prec, stream=stream)
        return self.gs.apply(yl.view(yl.shape[0], -1), GS_QT, stream=stream)


def cg_solve(prob: Problem, b, x=None, rtol=1e-10, max_it=20000, inner_prec=AX_FP64, inner_rtol=1e-6,
             max_outer=50, use_graph=True, refine=None, precond=AX_PRECOND_NONE, stream=None):
    """Solve A x = b by CG (inner_prec = AX_FP64) or mixed-precision iterative refinement
    (refine = AX_REFINE_RESTART, the default, or AX_REFINE_RELIABLE).  b [nrhs][n_global]
    float64 device.  Returns (x, report dict); raises AxError only on argument or launch errors
    (non-convergence and breakdown are reported in the dict)."""
    import torch
    nrhs = b.shape[0] if b.dim() == 2 else 1
    if x is None:
        x = torch.zeros_like(b)
    p = prob.c_struct()
    opts = AxCgOpts(rtol, max_it, inner_prec, inner_rtol, max_outer, None, 0, 1 if use_graph else 0,
                    AX_REFINE_RESTART if refine is None else refine, precond)
    nbytes = ctypes.c_size_t()
    _check(lib().cg_workspace_bytes(ctypes.byref(p), nrhs, ctypes.byref(opts), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=b.device)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = nbytes.value
    rep = AxCgReport()
    code = lib().cg_solve(ctypes.byref(p), nrhs, _dptr(b), _dptr(x), ctypes.byref(opts), ctypes.byref(rep),
                          _stream(stream))
    if code not in (AX_OK, AX_ERR_NOT_CONVERGED, AX_ERR_BREAKDOWN):
        _check(code)
    return x, {"status": _STATUS.get(code, code), "outer_it": rep.outer_it, "iterations": rep.inner_it_total,
               "rel_res_true": rep.rel_res_true, "seconds": rep.seconds}


class BatchedAxLocal:
    """AxLocal over many trilinear meshes (uneven E and N <= 9) in one persistent launch.

    meshes: list of (verts [E][8][3] float64 device tensor, Basis); X, Y: lists of device
    tensors [nrhs][E][N1^3] (float64 for AX_FP64, float32 for AX_FP32).  The work list and the
    X/Y pointers are uploaded once; launch() enqueues the single kernel (graph-capturable)."""

    def __init__(self, meshes, X, Y, prec=AX_FP64, device="cuda"):
        import torch
        n = len(meshes)
        self._keep = (meshes, X, Y)
        self.probs = (AxProblem * max(n, 1))()
        for q, (verts, basis) in enumerate(meshes):
            self.probs[q] = AxProblem(verts.shape[0], basis.N, AX_TRILINEAR, verts.data_ptr(), basis.D.ctypes.data,
                                      basis.xi.ctypes.data, basis.w.ctypes.data, 0, None, None, None, None)
        nrhs = X[0].shape[0] if n else 1
        nbytes = ctypes.c_size_t()
        _check(lib().ax_batched_workspace_bytes(n, self.probs, ctypes.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
        xs = (ctypes.c_void_p * max(n, 1))(*[x.data_ptr() for x in X])
        ys = (ctypes.c_void_p * max(n, 1))(*[y.data_ptr() for y in Y])
        self.plan = AxBatchPlan()
        _check(lib().ax_batched_prepare(n, self.probs, nrhs, prec, ctypes.cast(xs, ctypes.c_void_p),
                                        ctypes.cast(ys, ctypes.c_void_p), None, _dptr(self.ws), nbytes.value,
                                        ctypes.byref(self.plan)))

    def launch(self, stream=None):
        _check(lib().ax_local_batched(ctypes.byref(self.plan), _dptr(self.ws), _stream(stream)))


def item_shape_of(N1: int, variant: int, prec=AX_FP64) -> dict:
    """Work-group shape of the batched kernels of order N1 - 1 in a plan's shape variant (0 or 1
    the per-item shapes, 2 the tile kernel over the work list, 3 over mesh slices) and precision."""
    if int(variant) in (2, 3):
        t = AxTune(kernel=AX_KERNEL_TILE, tile_alt=int(variant) - 2, grid_mult=2)
    else:
        t = AxTune(kernel=AX_KERNEL_ITEM, item_alt=int(variant), grid_mult=2)
    saved = AxTune()
    L = lib()
    kind = AX_TUNE_BATCHED if N1 <= 10 else AX_TUNE_TRILINEAR
    _check(L.ax_tune_get(N1 - 1, kind, prec, ctypes.byref(saved)))
    try:
        _check(L.ax_tune_set(N1 - 1, kind, prec, ctypes.byref(t)))
        _check(L.ax_tune_get(N1 - 1, kind, prec, ctypes.byref(t)))
    finally:
        _check(L.ax_tune_set(N1 - 1, kind, prec, ctypes.byref(saved)))
    kernel = "item" if t.kernel_used != AX_KERNEL_TILE else ("tile slices" if int(variant) == 3 else "tile")
    return {"kernel": kernel, "elems_per_group": t.elems_per_group, "block": t.block}


def probe_copy(src, dst, stream=None):
    """dst = src with the library's copy probe (HBM bandwidth); both contiguous device tensors of
    the same byte size (a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().ax_probe_copy(_dptr(src), _dptr(dst), nbytes, _stream(stream)))


def probe_compute(kind, iters, out=None, stream=None):
    """One launch of an arithmetic probe loop; returns (out tensor, flops of the launch)."""
    import torch
    n = ctypes.c_size_t()
    _check(lib().ax_probe_compute_elems(ctypes.byref(n)))
    dt = torch.float64 if kind in (AX_PROBE_FMA_F64, AX_PROBE_MFMA_F64, AX_PROBE_MIX_F64) else torch.float32
    if out is None or out.numel() < n.value or out.dtype != dt:
        out = torch.empty(n.value, dtype=dt, device="cuda")
    fl = ctypes.c_double()
    _check(lib().ax_probe_compute(kind, iters, _dptr(out), ctypes.byref(fl), _stream(stream)))
    return out, fl.value


def batched_noalloc(meshes, X, Y, prec=AX_FP64, stream=None):
    """The batched AxLocal of BatchedAxLocal in one allocation-free call (ax_local_batched_noalloc):
    meshes as for BatchedAxLocal, X, Y lists of device tensors [nrhs][E][N1^3]."""
    n = len(meshes)
    probs = (AxProblem * max(n, 1))()
    for q, (verts, basis) in enumerate(meshes):
        probs[q] = AxProblem(verts.shape[0], basis.N, AX_TRILINEAR, verts.data_ptr(), basis.D.ctypes.data,
                             basis.xi.ctypes.data, basis.w.ctypes.data, 0, None, None, None, None)
    nrhs = X[0].shape[0] if n else 1
    xs = (ctypes.c_void_p * max(n, 1))(*[x.data_ptr() for x in X])
    ys = (ctypes.c_void_p * max(n, 1))(*[y.data_ptr() for y in Y])
    _check(lib().ax_local_batched_noalloc(n, probs, nrhs, prec, ctypes.cast(xs, ctypes.c_void_p),
                                          ctypes.cast(ys, ctypes.c_void_p), None, _stream(stream)))


def cg_solve_batched(meshes, gs: GatherScatter, b, x=None, rtol=1e-10, max_it=20000, inner_prec=AX_FP64,
                     inner_rtol=1e-6, max_outer=50, use_graph=True, refine=None, precond=AX_PRECOND_NONE,
                     stream=None):
    """CG / mixed refinement over the union of many trilinear meshes (block-diagonal system).
    meshes: list of (verts device tensor, Basis) in the order of the concatenated local vectors;
    gs: gather-scatter of the concatenated numbering; b [nrhs][n_global] float64 device."""
    import torch
    n = len(meshes)
    probs = (AxProblem * n)()
    for q, (verts, basis) in enumerate(meshes):
        probs[q] = AxProblem(verts.shape[0], basis.N, AX_TRILINEAR, verts.data_ptr(), basis.D.ctypes.data,
                             basis.xi.ctypes.data, basis.w.ctypes.data, 0, None, None, None, None)
    nrhs = b.shape[0] if b.dim() == 2 else 1
    if x is None:
        x = torch.zeros_like(b)
    opts = AxCgOpts(rtol, max_it, inner_prec, inner_rtol, max_outer, None, 0, 1 if use_graph else 0,
                    AX_REFINE_RESTART if refine is None else refine, precond)
    nbytes = ctypes.c_size_t()
    _check(lib().cg_batched_workspace_bytes(n, probs, gs.n_global, nrhs, ctypes.byref(opts), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=b.device)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = nbytes.value
    rep = AxCgReport()
    code = lib().cg_solve_batched(n, probs, gs.n_global, _dptr(gs.l2g), _dptr(gs.gptr), _dptr(gs.gidx),
                                  _dptr(gs.mask) if gs.mask is not None else None, nrhs, _dptr(b), _dptr(x),
                                  ctypes.byref(opts), ctypes.byref(rep), _stream(stream))
    if code not in (AX_OK, AX_ERR_NOT_CONVERGED, AX_ERR_BREAKDOWN):
        _check(code)
    return x, {"status": _STATUS.get(code, code), "outer_it": rep.outer_it, "iterations": rep.inner_it_total,
               "rel_res_true": rep.rel_res_true, "seconds": rep.seconds}
