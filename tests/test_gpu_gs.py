"""GPU gather-scatter (Q, Q^T, Q Q^T with a Dirichlet mask) against the oracle: bit-exact,
including the library's CSR inverse of the local-to-global map."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("N,grid", [(1, (2, 2, 2)), (3, (4, 3, 2)), (7, (3, 3, 3)), (4, (3, 1, 1))])
def test_gs_bitexact(ax, N, grid):
    import torch
    l2g, ng, mask = meshgen.global_numbering(*grid, N)
    gs = ax.GatherScatter(l2g, ng, mask)
    rng = np.random.default_rng(N)
    yl = rng.uniform(-1, 1, (2, l2g.size))
    xg = rng.uniform(-1, 1, (2, ng))
    qt = gs.apply(torch.from_numpy(yl).cuda(), ax.GS_QT).cpu().numpy()
    ref = oracle.gs_qt(l2g, ng, yl)
    ref[:, mask == 1] = 0.0
    assert np.array_equal(qt, ref)
    q = gs.apply(torch.from_numpy(xg).cuda(), ax.GS_Q).cpu().numpy()
    assert np.array_equal(q, oracle.gs_q(l2g, xg))
    qqt = gs.apply(torch.from_numpy(yl).cuda(), ax.GS_QQT).cpu().numpy()
    assert np.array_equal(qqt, oracle.gs_q(l2g, ref))
    # float32 path: same order of additions, so bit-exact against an FP32 replay
    yl32 = yl.astype(np.float32)
    qt32 = gs.apply(torch.from_numpy(yl32).cuda(), ax.GS_QT, use_mask=False).cpu().numpy()
    gptr, gidx = ax.gs_build_csr(l2g, ng)
    ref32 = np.zeros((2, ng), dtype=np.float32)
    for g in range(ng):
        s = np.zeros(2, dtype=np.float32)
        for p in range(gptr[g], gptr[g + 1]):
            s = (s + yl32[:, gidx[p]]).astype(np.float32)
        ref32[:, g] = s
    assert np.array_equal(qt32, ref32)
