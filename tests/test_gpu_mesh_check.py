"""GPU checks of the mesh validity call (det J of the trilinear map, Eq. 8-9, at every GLL node):
the smallest det J equals the oracle's, and inverted, collapsed, partly folded and non-finite
elements are named."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import report
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


def _oracle_dets(verts, N):
    xi, _, _ = oracle.gll(N)
    return np.linalg.det(oracle.jacobians(verts, N, xi))   # [E][N1^3]


def _run(ax, verts, N):
    import torch
    return ax.check_mesh(torch.from_numpy(np.ascontiguousarray(verts)).cuda(), ax.Basis(N))


@pytest.mark.parametrize("alpha", [0.2, 0.3])
@pytest.mark.parametrize("N", [1, 3, 7, 15])
def test_jittered_mesh(ax, N, alpha):
    """Random vertex jitter of 20 % of the spacing keeps every element valid; at 30 % some seeds
    fold an element near a node (det J < 0 there): the first such element is named either way."""
    m = meshgen.jittered_hex(8, 6, 5, alpha=alpha, seed=40 + N)
    bad, dmin = _run(ax, m.verts, N)
    ref = _oracle_dets(m.verts, N)
    flagged = np.flatnonzero((ref <= 0).any(axis=1))
    report("check_mesh", N=N, alpha=alpha, bad=bad, min_det=dmin, oracle=ref.min(), oracle_bad=flagged[:4].tolist())
    assert bad == (flagged[0] if flagged.size else -1)
    if alpha == 0.2:
        assert bad == -1
    assert abs(dmin - ref.min()) <= 1e-13 * abs(ref).max()


def test_parallelepipeds(ax):
    m, _ = meshgen.parallelepiped_hex(5, 4, 3, seed=3)
    bad, dmin = _run(ax, m.verts, 5)
    assert bad == -1 and abs(dmin - _oracle_dets(m.verts, 5).min()) <= 1e-13 * abs(dmin)
    v = m.verts.copy()
    v[17] = v[17][[1, 0, 3, 2, 5, 4, 7, 6]]     # mirror element 17 in r: a left-handed map
    bad, dmin = _run(ax, v, 5)
    assert bad == 17 and dmin < 0


@pytest.mark.parametrize("N", [3, 7])
def test_bad_elements_named(ax, N):
    m = meshgen.jittered_hex(6, 5, 4, alpha=0.2, seed=9)
    v = m.verts.copy()
    v[40] = v[40][[1, 0, 3, 2, 5, 4, 7, 6]]     # inverted: det J < 0 at every node
    v[23, 4:] = v[23, :4]                       # collapsed in t: det J = 0 at every node
    # fold one corner: vertex 7 pulled past the element's centre, so det J changes sign inside
    v[95, 7] = v[95, 0] + 0.05 * (v[95, 7] - v[95, 0])
    ref = _oracle_dets(v, N)
    assert (ref[95] > 0).any() and (ref[95] < 0).any()
    assert (ref[23] == 0).all() and (ref[40] < 0).all()
    assert np.flatnonzero((ref <= 0).any(axis=1)).tolist() == [23, 40, 95]
    bad, dmin = _run(ax, v, N)
    report("check_mesh_bad", N=N, bad=bad, min_det=dmin, oracle=ref.min())
    assert bad == 23
    assert abs(dmin - ref.min()) <= 1e-13 * abs(ref).max()
    # the raw call returns AX_ERR_ARG and names the element
    import torch
    L = ax.lib()
    b = ax.Basis(N)
    dv = torch.from_numpy(v).cuda()
    out = ctypes.c_int64(0)
    code = L.ax_check_mesh(v.shape[0], N, ax._dptr(dv), ax._np_ptr(b.xi), ctypes.byref(out), None, None)
    assert code == ax.AX_ERR_ARG and out.value == 23
    assert "element 23" in L.ax_last_error().decode()
    # only the folded element left: it is found although most of its nodes are valid
    v2 = m.verts.copy()
    v2[95] = v[95]
    bad, _ = _run(ax, v2, N)
    assert bad == 95


def test_non_finite_vertex(ax):
    m = meshgen.jittered_hex(4, 4, 4, alpha=0.1, seed=1)
    v = m.verts.copy()
    v[63, 2, 1] = np.nan
    bad, dmin = _run(ax, v, 3)
    assert bad == 63
    assert np.isfinite(dmin) and dmin > 0
    v = m.verts.copy()
    v[5, 0, 0] = np.inf
    assert _run(ax, v, 3)[0] == 5


def test_empty_and_large(ax):
    import torch
    assert ax.check_mesh(torch.zeros((0, 8, 3), dtype=torch.float64, device="cuda"), ax.Basis(7)) == (-1, np.inf)
    # the headline mesh (32^3 trilinear elements at N = 7): valid, smallest det matches the oracle
    m = meshgen.jittered_hex(32, 32, 32, alpha=0.15, seed=7)
    bad, dmin = _run(ax, m.verts, 7)
    ref = min(_oracle_dets(m.verts[e0:e0 + 2048], 7).min() for e0 in range(0, m.E, 2048))
    report("check_mesh_32^3", bad=bad, min_det=dmin, oracle=ref)
    assert bad == -1 and abs(dmin - ref) <= 1e-13 * ref
