"""GPU parity of the gathering operator Y = AxLocal(Q Xg) (the CG solver's operator application,
the gather of Eq. 1 fused into the load) against the oracle's Q then AxLocal (Eq. 3), and bit for
bit against the two-step gs_assemble(GS_Q) + ax_local path.  Small meshes over every order; the
CG workload itself (N = 7, 32^3, 11.4 M global nodes) on sampled elements."""
import numpy as np
import pytest

import oracle
from gpu_util import U32, check_bound, check_fp64, cond_j_per_element, fp32_bound, report, sample_elements
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("geom", ["tri", "para"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 9, 11, 12, 15])
def test_gathered_small(ax, N, prec, geom):
    import torch
    P = ax.AX_FP64 if prec == "fp64" else ax.AX_FP32
    dims = (4, 3, 3)
    if geom == "tri":
        m = meshgen.jittered_hex(*dims, alpha=0.15, seed=700 + N)
    else:
        m, _ = meshgen.parallelepiped_hex(*dims, seed=N)
    l2g, ng, _ = meshgen.global_numbering(*dims, N)
    rng = np.random.default_rng(N)
    Xg = rng.uniform(-1, 1, (2, ng))
    b = ax.Basis(N)
    V = _dev(m.verts)
    geo = V if geom == "tri" else ax.parallelepiped_factors(V)
    G_ = ax.AX_TRILINEAR if geom == "tri" else ax.AX_PARALLELEPIPED
    T = torch.float64 if P == ax.AX_FP64 else torch.float32
    Xgd = _dev(Xg).to(T)
    Y = ax.ax_local_gathered(Xgd, _dev(l2g), geo, b, G_, P)
    # two-step path: Q on the device, then the streaming operator: bit for bit the same
    Xl = torch.stack([Xgd[c][_dev(l2g).long()] for c in range(2)]).reshape(2, m.E, -1).contiguous()
    Y2 = ax.ax_local(Xl, geo, b, G_, P)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y2)
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    xs = Xg.astype(np.float32).astype(np.float64) if P == ax.AX_FP32 else Xg
    Xloc = np.stack([oracle.gs_q(l2g, xs[c]) for c in range(2)]).reshape(2, m.E, -1)
    Yref, env = oracle.ax_local(D, G, Xloc), oracle.ax_envelope(D, G, Xloc)
    tag = f"gathered N={N} {prec} {geom}"
    if P == ax.AX_FP64:
        check_fp64(Y.cpu().numpy(), Yref, env, tag=tag)
    else:
        check_bound(Y.double().cpu().numpy(), Yref, env, fp32_bound(N, cond_j_per_element(m.verts, N))[None, :, None],
                    tag=tag)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gathered_cg_workload(ax, prec):
    """The CG's own operator size: N = 7, 32^3 elements, 11.4 M global nodes, sampled elements
    (every work-group takes several elements; the last ones are the ragged tail)."""
    import torch
    P = ax.AX_FP64 if prec == "fp64" else ax.AX_FP32
    N, dims = 7, (32, 32, 32)
    m = meshgen.jittered_hex(*dims, alpha=0.10, seed=4)
    l2g, ng, _ = meshgen.global_numbering(*dims, N)
    T = torch.float64 if P == ax.AX_FP64 else torch.float32
    Xgd = meshgen.random_global_device(ng, np.zeros(ng, np.uint8), 1, seed=3, device="cuda").to(T)
    b = ax.Basis(N)
    Y = ax.ax_local_gathered(Xgd, _dev(l2g), _dev(m.verts), b, ax.AX_TRILINEAR, P)
    torch.cuda.synchronize()
    sel = sample_elements(m.E, 64, seed=11)
    xg = Xgd.double().cpu().numpy()[0]
    NP = (N + 1) ** 3
    Xloc = xg[l2g.reshape(m.E, NP)[sel]][None]
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts[sel], N, xi, w)
    Yref, env = oracle.ax_local(D, G, Xloc), oracle.ax_envelope(D, G, Xloc)
    Ys = Y[:, torch.from_numpy(sel).cuda()].double().cpu().numpy()
    tag = f"gathered CG workload {prec} ({len(sel)} sampled elements)"
    if P == ax.AX_FP64:
        check_fp64(Ys, Yref, env, tag=tag)
    else:
        check_bound(Ys, Yref, env, fp32_bound(N, cond_j_per_element(m.verts[sel], N))[None, :, None], tag=tag)
    report("gathered_cg_workload", prec=prec, n_global=ng, E=m.E)


def test_gathered_validation(ax):
    import ctypes
    L = ax.lib()
    b = ax.Basis(3)
    D, xi, w = ax._np_ptr(b.D), ax._np_ptr(b.xi), ax._np_ptr(b.w)
    v = ctypes.c_void_p
    assert L.ax_local_gathered(4, 3, 0, v(8), D, xi, w, 1, ax.AX_FP64, None, 10, v(16), v(24), None) == ax.AX_ERR_ARG
    assert L.ax_local_gathered(4, 3, 0, v(8), D, xi, w, 1, ax.AX_FP64, v(8), 0, v(16), v(24), None) == ax.AX_ERR_ARG
    assert L.ax_local_gathered(4, 3, 0, v(8), D, xi, w, 1, ax.AX_FP16_ACC32, v(8), 10, v(16), v(24),
                               None) == ax.AX_ERR_UNSUPPORTED
    assert L.ax_local_gathered(4, 3, 0, v(8), D, xi, w, 1, ax.AX_FP64, v(8), 10, v(16), v(16), None) == ax.AX_ERR_ARG
    assert L.ax_local_gathered(0, 3, 0, None, D, xi, w, 1, ax.AX_FP64, None, 10, None, None, None) == ax.AX_OK


def _energy_factor(N, kappa):
    """Bound factor of the FP32 energy sum_e X_e^T Y_e, in units of sum_e |X_e|^T env_e =
    sum over nodes of (|D||X|)^T |G| (|D||X|): each node's (D X)^T G (D X) carries the operator's
    FP32 forward error (fp32_bound) plus N1 u32 for the FP32 sum over an element column; the
    further sums are FP64."""
    return fp32_bound(N, kappa) + (N + 1) * U32


def _energy_ref(D, G, Xloc):
    """sum_e X_e^T AxLocal(X_e) and its envelope sum_e |X_e|^T env_e from the oracle (Eq. 3)."""
    Yref, env = oracle.ax_local(D, G, Xloc), oracle.ax_envelope(D, G, Xloc)
    return float(np.sum(Xloc * Yref)), float(np.sum(np.abs(Xloc) * env)), Yref, env


@pytest.mark.parametrize("geom", ["tri", "para"])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 9, 11, 12, 15])
def test_gathered_energy_small(ax, N, geom):
    """The CG's FP32 inner operator with p^T A p summed in the kernel: Y against the oracle under
    the FP32 bound, the energy against sum_e X_e^T AxLocal(X_e) under its own bound.  The orders
    cover one- and several-wave work-groups (the cross-wave sum of the energies)."""
    import torch
    dims = (4, 3, 3)
    if geom == "tri":
        m = meshgen.jittered_hex(*dims, alpha=0.15, seed=900 + N)
    else:
        m, _ = meshgen.parallelepiped_hex(*dims, seed=N + 50)
    l2g, ng, _ = meshgen.global_numbering(*dims, N)
    xg = np.random.default_rng(N + 5).uniform(-1, 1, ng).astype(np.float32)
    b = ax.Basis(N)
    V = _dev(m.verts)
    geo = V if geom == "tri" else ax.parallelepiped_factors(V)
    G_ = ax.AX_TRILINEAR if geom == "tri" else ax.AX_PARALLELEPIPED
    Y, en = ax.ax_local_gathered_energy(_dev(xg), _dev(l2g), geo, b, G_)
    torch.cuda.synchronize()
    xi, w, D = oracle.gll(N)
    G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
    Xloc = oracle.gs_q(l2g, xg.astype(np.float64)).reshape(1, m.E, -1)
    e_ref, e_env, Yref, env = _energy_ref(D, G, Xloc)
    kappa = cond_j_per_element(m.verts, N)
    tag = f"gathered energy N={N} {geom}"
    check_bound(Y.double().cpu().numpy()[None], Yref, env, fp32_bound(N, kappa)[None, :, None], tag=tag)
    err = abs(float(en.item()) - e_ref)
    bound = float(_energy_factor(N, kappa.max())) * e_env
    report(tag + " energy", energy=e_ref, err_over_env=err / e_env, fraction_of_bound=err / bound)
    assert e_ref > 0.0
    assert err <= bound, (en.item(), e_ref, err, bound)


def test_gathered_energy_cg_workload(ax):
    """The FP32 inner operator at the CG's size (N = 7, 32^3, 11.4 M global nodes; every
    work-group takes several elements): the energy over the whole mesh against the oracle,
    evaluated in element chunks, and Y on sampled elements."""
    import torch
    N, dims = 7, (32, 32, 32)
    m = meshgen.jittered_hex(*dims, alpha=0.10, seed=4)
    l2g, ng, _ = meshgen.global_numbering(*dims, N)
    xg = np.random.default_rng(17).uniform(-1, 1, ng).astype(np.float32)
    b = ax.Basis(N)
    Y, en = ax.ax_local_gathered_energy(_dev(xg), _dev(l2g), _dev(m.verts), b, ax.AX_TRILINEAR)
    torch.cuda.synchronize()
    xi, w, D = oracle.gll(N)
    NP = (N + 1) ** 3
    L = l2g.reshape(m.E, NP)
    e_ref = e_env = 0.0
    kmax = 1.0
    for e0 in range(0, m.E, 4096):
        sl = slice(e0, min(e0 + 4096, m.E))
        G, _, _ = oracle.geom_factors(m.verts[sl], N, xi, w)
        er, ee, _, _ = _energy_ref(D, G, xg.astype(np.float64)[L[sl]][None])
        e_ref += er
        e_env += ee
        kmax = max(kmax, float(cond_j_per_element(m.verts[sl], N).max()))
    sel = sample_elements(m.E, 64, seed=12)
    kappa = cond_j_per_element(m.verts[sel], N)
    G, _, _ = oracle.geom_factors(m.verts[sel], N, xi, w)
    Xs = xg.astype(np.float64)[L[sel]][None]
    Yref, env = oracle.ax_local(D, G, Xs), oracle.ax_envelope(D, G, Xs)
    check_bound(Y[torch.from_numpy(sel).cuda()].double().cpu().numpy()[None], Yref, env,
                fp32_bound(N, kappa)[None, :, None], tag="gathered energy CG workload (sampled Y)")
    err = abs(float(en.item()) - e_ref)
    bound = float(_energy_factor(N, kmax)) * e_env
    report("gathered energy CG workload", energy=e_ref, err_over_env=err / e_env, fraction_of_bound=err / bound)
    assert err <= bound, (en.item(), e_ref, err, bound)
