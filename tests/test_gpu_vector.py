"""GPU parity of the vector-field operator (n_col = 3, component-interleaved [E][3][N1^3], one
geometric set-up per element shared by the three components) against the oracle, which applies
Eq. 3 to the three components as three columns."""
import numpy as np
import pytest

import oracle
from gpu_util import check_bound, check_fp64, cond_j_per_element, fp32_bound, sample_elements
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


def _columns(Xv):
    """[E][3][N1^3] -> the oracle's [3][E][N1^3]."""
    return np.ascontiguousarray(np.transpose(Xv, (1, 0, 2)))


@pytest.mark.parametrize("geom", ["tri", "para"])
@pytest.mark.parametrize("N", [1, 3, 5, 7, 8, 11, 15])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vector_field(ax, N, geom, prec):
    import torch
    if geom == "tri":
        m = meshgen.jittered_hex(3, 3, 2, alpha=0.15, seed=500 + N)
    else:
        m, _ = meshgen.parallelepiped_hex(3, 2, 3, seed=N)
    NP = (N + 1) ** 3
    Xv = meshgen.random_nodal(m.E, N, nrhs=3, seed=N).reshape(m.E, 3, NP)
    if prec == "fp32":
        Xv = Xv.astype(np.float32).astype(np.float64)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Xc = _columns(Xv)
    Yref = oracle.ax_local(D, G, Xc)
    env = oracle.ax_envelope(D, G, Xc)
    b = ax.Basis(N)
    V = torch.from_numpy(m.verts).cuda()
    geo = V if geom == "tri" else ax.parallelepiped_factors(V)
    g = ax.AX_TRILINEAR if geom == "tri" else ax.AX_PARALLELEPIPED
    if prec == "fp64":
        Y = ax.ax_local_vector(torch.from_numpy(Xv).cuda(), geo, b, g, ax.AX_FP64).cpu().numpy()
        check_fp64(_columns(Y), Yref, env, tag=f"vector {geom} fp64 N={N}")
    else:
        Y = ax.ax_local_vector(torch.from_numpy(Xv.astype(np.float32)).cuda(), geo, b, g, ax.AX_FP32).cpu().numpy()
        kappa = cond_j_per_element(m.verts, N)[None, :, None]
        check_bound(_columns(Y).astype(np.float64), Yref, env, fp32_bound(N, kappa), tag=f"vector {geom} fp32 N={N}")


def test_vector_field_full_size_sampled(ax):
    """N = 7 on 32^3 trilinear elements (the benchmark's vector-field leg), sampled elements."""
    import torch
    N = 7
    m = meshgen.jittered_hex(32, 32, 32, alpha=0.15, seed=N)
    NP = (N + 1) ** 3
    Xv = meshgen.random_nodal(m.E, N, nrhs=3, seed=N + 3).reshape(m.E, 3, NP)
    b = ax.Basis(N)
    Y = ax.ax_local_vector(torch.from_numpy(Xv).cuda(), torch.from_numpy(m.verts).cuda(), b)
    sample = sample_elements(m.E, seed=3)
    Ys = Y[torch.from_numpy(sample).cuda()].cpu().numpy()
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts[sample], N, xi, w)
    Xc = _columns(Xv[sample])
    check_fp64(_columns(Ys), oracle.ax_local(D, G, Xc), oracle.ax_envelope(D, G, Xc), tag="vector full size fp64 N=7")


def test_vector_field_rejects_fp16(ax):
    import torch
    b = ax.Basis(7)
    m = meshgen.jittered_hex(1, 1, 1)
    X = torch.zeros((1, 3, 512), dtype=torch.float32, device="cuda")
    with pytest.raises(ax.AxError) as ei:
        ax.ax_local_vector(X, torch.from_numpy(m.verts).cuda(), b, ax.AX_TRILINEAR, ax.AX_FP16_ACC32)
    assert ei.value.code == ax.AX_ERR_UNSUPPORTED
