"""Seeded synthetic inputs: structured hexahedral meshes, their global node numbering and
random nodal vectors.

This module only *generates inputs*. It evaluates nothing of the method itself: no basis
constants, no Jacobians, no geometric factors, no operator. Both the HIP path and the CPU
oracle consume the arrays it returns, so every comparison between them starts from identical
bytes.

Conventions (all fixed by the paper's notation):

* Element ``e = ex + nx*(ey + ny*ez)`` of an ``nx x ny x nz`` grid.
* Vertex order inside an element is the tensor (lexicographic) order of the trilinear map in
  Kronecker form (Sec. 3.3, Eq. 8): vertex ``v = a + 2b + 4c`` sits at reference corner
  ``(r, s, t) = (2a-1, 2b-1, 2c-1)``.  It is *not* the VTK/Gmsh counter-clockwise order.
* Local node ``[i, j, k]`` of element ``e`` has local index ``i + j*N1 + k*N1**2`` (Sec. 2.2,
  index rule stated with Alg. 1), ``N1 = N + 1``; local vectors are ``[nrhs][E][N1**3]``.
* The global-to-local map Q (Sec. 2.1) is stored as ``l2g[e*N1**3 + l] = g``.  For a
  structured grid the global node ids are lexicographic over the ``(nx*N+1) x (ny*N+1) x
  (nz*N+1)`` lattice of GLL nodes, ``g = I + J*Gx + K*Gx*Gy``.

Recipes (the paper gives none; these are the synthetic stand-ins for its box meshes):

* Jitter ``alpha``: every grid vertex not on the boundary of the unit cube moves by an
  independent ``U(-alpha, alpha) * h_d`` per coordinate ``d``; boundary vertices stay put so the
  domain stays the unit cube.  Draw: ``default_rng(seed).uniform(-alpha, alpha,
  (nz+1, ny+1, nx+1, 3))`` in C order, boundary rows zeroed.
* Parallelepipeds: the grid of the unit cube is mapped by ``M = U diag(1, s2, s3) V^T`` with
  ``U, V`` orthogonal (QR of seeded Gaussians, sign-fixed, det +1), ``s3 ~ U(1,4)``,
  ``s2 ~ U(1, s3)``, so ``cond(M) <= 4`` and every element is the same parallelepiped.
* Nodal vectors: ``default_rng([seed, 1]).uniform(-1, 1, nrhs*E*N1**3)``.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class HexMesh:
    """A structured hex mesh of ``nx*ny*nz`` elements.

    ``verts``: float64 ``[E][8][3]``, tensor vertex order.
    ``nx, ny, nz``: grid size; ``E = nx*ny*nz``.
    """

    nx: int
    ny: int
    nz: int
    verts: np.ndarray

    @property
    def E(self) -> int:
        return self.nx * self.ny * self.nz


def _grid_points(nx: int, ny: int, nz: int) -> np.ndarray:
    """Grid vertices of the unit cube, shape (nz+1, ny+1, nx+1, 3), coordinates (x, y, z)."""
    x = np.linspace(0.0, 1.0, nx + 1)
    y = np.linspace(0.0, 1.0, ny + 1)
    z = np.linspace(0.0, 1.0, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def _gather_elements(P: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Collect the 8 corner points of every element in tensor order v = a + 2b + 4c."""
    verts = np.empty((nz, ny, nx, 8, 3), dtype=np.float64)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                verts[:, :, :, a + 2 * b + 4 * c, :] = P[c:c + nz, b:b + ny, a:a + nx, :]
    return np.ascontiguousarray(verts.reshape(nx * ny * nz, 8, 3))


def jittered_hex(nx: int, ny: int, nz: int, alpha: float = 0.0, seed: int = 0) -> HexMesh:
    """Unit-cube grid with interior vertices jittered by ``U(-alpha, alpha) * h`` per axis."""
    P = _grid_points(nx, ny, nz)
    if alpha > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-alpha, alpha, size=(nz + 1, ny + 1, nx + 1, 3))
        d[0, :, :, :] = 0.0
        d[-1, :, :, :] = 0.0
        d[:, 0, :, :] = 0.0
        d[:, -1, :, :] = 0.0
        d[:, :, 0, :] = 0.0
        d[:, :, -1, :] = 0.0
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        P = P + d * h
    return HexMesh(nx, ny, nz, _gather_elements(P, nx, ny, nz))


def random_affine(seed: int, max_cond: float = 4.0) -> np.ndarray:
    """Seeded 3x3 map ``U diag(1, s2, s3) V^T`` with det > 0 and condition number <= max_cond."""
    rng = np.random.default_rng(seed)

    def rot() -> np.ndarray:
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        return q

    U = rot()
    V = rot()
    s3 = rng.uniform(1.0, max_cond)
    s2 = rng.uniform(1.0, s3)
    return U @ np.diag([1.0, s2, s3]) @ V.T


def parallelepiped_hex(nx: int, ny: int, nz: int, seed: int = 2, max_cond: float = 4.0):
    """Unit-cube grid mapped by a seeded shear/scale matrix M: every element is the same
    parallelepiped.  Returns (mesh, M)."""
    M = random_affine(seed, max_cond)
    P = _grid_points(nx, ny, nz) @ M.T
    return HexMesh(nx, ny, nz, _gather_elements(P, nx, ny, nz)), M


def chain_hex(n: int, h: float = 1.0) -> HexMesh:
    """``n`` unit cubes in a row along x (a face-connected chain)."""
    P = _grid_points(n, 1, 1)
    P = P * np.array([n * h, h, h])
    return HexMesh(n, 1, 1, _gather_elements(P, n, 1, 1))


def box_element(hx: float, hy: float, hz: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """One axis-aligned box element, vertices ``[1][8][3]`` in tensor order."""
    v = np.empty((1, 8, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                v[0, a + 2 * b + 4 * c] = (origin[0] + a * hx, origin[1] + b * hy, origin[2] + c * hz)
    return v


def global_numbering(nx: int, ny: int, nz: int, N: int, order: str = "lexicographic"):
    """Global numbering of the GLL nodes of an nx x ny x nz box of hexahedra.

    ``order="lexicographic"`` (default) numbers the nodes of the global
    (nx N + 1)(ny N + 1)(nz N + 1) grid x-fastest; ``order="element"`` renumbers them by first
    appearance in the local (element-major) order, so that the new nodes of each element are
    consecutive.
    Returns ``(l2g, n_global, mask)``: ``l2g`` int32 ``[E*N1**3]``; ``mask`` uint8
    ``[n_global]``, 1 on nodes of the boundary of the box (homogeneous Dirichlet).
    """
    if order not in ("element", "lexicographic"):
        raise ValueError(f"unknown numbering order {order!r}")
    N1 = N + 1
    Gx, Gy, Gz = nx * N + 1, ny * N + 1, nz * N + 1
    n_global = Gx * Gy * Gz
    if n_global >= 2**31:
        raise ValueError("global node count exceeds int32")
    i = np.arange(N1)
    ex = np.arange(nx)
    ey = np.arange(ny)
    ez = np.arange(nz)
    # shape (nz, ny, nx, N1[k], N1[j], N1[i])
    I = (ex[None, None, :, None, None, None] * N + i[None, None, None, None, None, :])
    J = (ey[None, :, None, None, None, None] * N + i[None, None, None, None, :, None])
    K = (ez[:, None, None, None, None, None] * N + i[None, None, None, :, None, None])
    g = I + J * Gx + K * (Gx * Gy)
    l2g = np.ascontiguousarray(g.reshape(-1).astype(np.int32))
    gI = np.arange(n_global) % Gx
    gJ = (np.arange(n_global) // Gx) % Gy
    gK = np.arange(n_global) // (Gx * Gy)
    mask = ((gI == 0) | (gI == Gx - 1) | (gJ == 0) | (gJ == Gy - 1) | (gK == 0) | (gK == Gz - 1))
    mask = mask.astype(np.uint8)
    if order == "element":
        l2g, mask = first_touch(l2g, n_global, mask)
    return l2g, n_global, mask


def first_touch(l2g: np.ndarray, n_global: int, mask: np.ndarray):
    """Renumber global nodes by their first appearance in ``l2g``; returns (l2g', mask')."""
    _, first = np.unique(l2g, return_index=True)
    new_id = np.empty(n_global, dtype=np.int64)
    new_id[np.argsort(first, kind="stable")] = np.arange(n_global)
    mask_new = np.empty_like(mask)
    mask_new[new_id] = mask
    return np.ascontiguousarray(new_id[l2g].astype(np.int32)), mask_new


def chain_numbering(n: int, N: int):
    """Global numbering of an ``n``-element chain (same lexicographic rule)."""
    return global_numbering(n, 1, 1, N)


def random_nodal(E: int, N: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """X ~ U[-1, 1] per local node, shape ``[nrhs][E][N1**3]`` float64."""
    N1 = N + 1
    rng = np.random.default_rng([seed, 1])
    return rng.uniform(-1.0, 1.0, nrhs * E * N1**3).reshape(nrhs, E, N1**3)


def grid_for_nodes(N: int, target_nodes: int = 1 << 24):
    """A near-cubic ``(nx, ny, nz)`` with ``E*(N+1)**3`` close to ``target_nodes``."""
    E_target = target_nodes / (N + 1) ** 3
    best = None
    base = int(round(E_target ** (1.0 / 3.0)))
    for nx in range(max(1, base - 2), base + 3):
        for ny in range(max(1, base - 2), base + 3):
            for nz in range(max(1, base - 2), base + 3):
                E = nx * ny * nz
                err = abs(E - E_target)
                key = (err, max(nx, ny, nz) - min(nx, ny, nz))
                if best is None or key < best[0]:
                    best = (key, (nx, ny, nz))
    return best[1]


# The batched workload: many independent meshes of uneven size and order.
@dataclass
class BatchSpec:
    N: int
    nx: int
    ny: int
    nz: int
    seed: int


def batch_specs(n_mesh: int = 64, e_lo: int = 512, e_hi: int = 32768,
                orders=(3, 5, 7, 9), seed: int = 1) -> list:
    """Draw ``n_mesh`` (N, grid) pairs: E ~ U[e_lo, e_hi] rounded to a near-cubic grid,
    N uniform over ``orders``."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_mesh):
        E = int(rng.integers(e_lo, e_hi + 1))
        N = int(rng.choice(np.asarray(orders)))
        nx = max(1, int(round(E ** (1.0 / 3.0))))
        ny = max(1, int(round((E / nx) ** 0.5)))
        nz = max(1, int(round(E / (nx * ny))))
        out.append(BatchSpec(N, nx, ny, nz, seed * 1000 + m))
    return out


def concat_numbering(parts):
    """Concatenate per-mesh numberings [(l2g, n_global, mask), ...] into one index space (mesh
    after mesh, global ids offset by the preceding meshes' node counts).  Returns
    (l2g, n_global, mask, local_offsets, global_offsets)."""
    l2gs, masks, loff, goff = [], [], [0], [0]
    for l2g, ng, mask in parts:
        l2gs.append(l2g.astype(np.int64) + goff[-1])
        masks.append(mask)
        loff.append(loff[-1] + l2g.size)
        goff.append(goff[-1] + ng)
    if goff[-1] >= 2**31:
        raise ValueError("union node count exceeds int32")
    return (np.concatenate(l2gs).astype(np.int32), goff[-1], np.concatenate(masks),
            np.array(loff), np.array(goff))


def random_nodal_device(E: int, N: int, nrhs: int = 1, seed: int = 0, device="cuda", dtype=None):
    """X ~ U[-1, 1] per local node generated on the device by torch's seeded generator (for
    workloads too large to draw on the host); shape ``[nrhs][E][N1**3]``."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    dtype = dtype or torch.float64
    x = torch.rand((nrhs, E, (N + 1) ** 3), generator=g, device=device, dtype=dtype)
    return x.mul_(2.0).sub_(1.0)


def random_global_device(n_global: int, mask: np.ndarray, nrhs: int = 1, seed: int = 0, device="cuda"):
    """b ~ U[-1, 1] per global node (float64, on the device, torch's seeded generator), zero on
    the Dirichlet mask; shape ``[nrhs][n_global]``."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    b = torch.rand((nrhs, n_global), generator=g, device=device, dtype=torch.float64).mul_(2.0).sub_(1.0)
    b[:, torch.from_numpy(np.asarray(mask, dtype=bool)).to(device)] = 0.0
    return b
