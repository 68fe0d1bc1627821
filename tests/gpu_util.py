"""Helpers for the GPU parity tests: tolerances derived from the arithmetic, plus the device
set-up.  The oracle supplies every expected value."""
import numpy as np

import oracle

U64 = 2.0**-53
U32 = 2.0**-24

# FP64 bar (the relative 1e-12 of the target) applied both normwise and entrywise against the
# error envelope env = |D|^T |G| |D| |X| (entrywise relative error is meaningless where A 1 = 0
# makes an entry cancel).
TOL64 = 1e-12


def report(tag, **vals):
    """One line per bound check with the observed values (collected from the GPU test logs)."""
    txt = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items())
    print(f"[parity] {tag} {txt}", flush=True)


def check_fp64(Y, Yref, env, tol=TOL64, tag=""):
    Y = np.asarray(Y, dtype=np.float64).reshape(Yref.shape)
    d = np.abs(Y - Yref)
    nrm = np.linalg.norm(d) / max(np.linalg.norm(Yref), 1e-300)
    ent = (d / np.maximum(env, 1e-300)).max()
    report(tag or "fp64", normwise=float(nrm), max_err_over_env=float(ent), bar=tol)
    assert nrm <= tol, f"normwise rel err {nrm:.3e} > {tol}"
    assert ent <= tol, f"entrywise err / envelope {ent:.3e} > {tol}"
    return nrm, ent


def max_cond_j(verts, N):
    """Largest 2-norm condition number of the Jacobian over all GLL nodes (oracle Jacobian)."""
    xi, _, _ = oracle.gll(N)
    k = 1.0
    for e in range(verts.shape[0]):
        for kk in range(N + 1):
            for j in range(N + 1):
                for i in range(N + 1):
                    J = oracle.jacobian(verts[e], xi[i], xi[j], xi[kk])
                    k = max(k, np.linalg.cond(J))
    return k


def fp32_bound(N, kappa):
    """Forward-error bound factor of the FP32 kernel, in units of u32 * env: 2 N1 for the two
    length-N1 contractions per direction, 8 for D's rounding, the 3-term sums and the scaling,
    and 8 kappa^2 for forming adj(J^T J) / det J in single precision."""
    N1 = N + 1
    return (2 * N1 + 8 + 8 * kappa**2) * U32


def check_bound(Y, Yref, env, factor, tag=""):
    """|Y - Yref| <= factor * env entrywise; `factor` may be a scalar or broadcast per element."""
    Y = np.asarray(Y, dtype=np.float64).reshape(Yref.shape)
    rel = np.abs(Y - Yref) / np.maximum(env, 1e-300)
    ratio = float(rel.max())
    used = float((rel / np.broadcast_to(factor, rel.shape)).max())
    report(tag or "bound", max_err_over_env=ratio, max_fraction_of_bound=used,
           bound=float(np.max(factor)))
    assert used <= 1.0, f"max |dY|/env = {ratio:.3e} exceeds the bound ({used:.3f} of it)"
    return ratio


def cond_j_per_element(verts, N):
    """Largest 2-norm condition number of the Jacobian over the GLL nodes of each element
    (oracle Jacobian), shape [E]."""
    xi, _, _ = oracle.gll(N)
    J = oracle.jacobians(verts, N, xi)
    return np.linalg.cond(J.reshape(-1, 3, 3)).reshape(J.shape[:2]).max(axis=1)


def sample_elements(E, n=61, seed=0):
    """A seeded sample of element ids: n random ones plus the first two and the last five (the
    ragged tail of the last element group)."""
    rng = np.random.default_rng(seed)
    tail = np.arange(max(E - 5, 0), E)
    pick = rng.choice(E, min(n, E), replace=False)
    return np.unique(np.concatenate([pick, [0, min(1, E - 1)], tail]))
