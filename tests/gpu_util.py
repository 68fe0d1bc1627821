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


def check_fp64(Y, Yref, env, tol=TOL64):
    Y = np.asarray(Y, dtype=np.float64).reshape(Yref.shape)
    d = np.abs(Y - Yref)
    nrm = np.linalg.norm(d) / max(np.linalg.norm(Yref), 1e-300)
    ent = (d / np.maximum(env, 1e-300)).max()
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


def check_bound(Y, Yref, env, factor):
    Y = np.asarray(Y, dtype=np.float64).reshape(Yref.shape)
    ratio = (np.abs(Y - Yref) / np.maximum(env, 1e-300)).max()
    assert ratio <= factor, f"max |dY|/env = {ratio:.3e} > bound {factor:.3e}"
    return ratio
