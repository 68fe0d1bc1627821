"""Cases run twice by test_gpu_lds_poison.py: once on the release library in the test process and
once, as a script, in a child process on the LDS-poisoned debug build (AXHOSFEM_LIB).  Every kernel
family that holds LDS is covered: the per-order AxLocal kernels (on-the-fly trilinear and
parallelepiped, stored, partial, Helmholtz, vector; FP64, FP32 and the FP16 inner operator) and the
batched kernels.  Meshes are small but span several work-groups and a ragged last one.

Usage as a script: python tests/lds_poison_cases.py OUT.npz  (writes every case's output)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def run_all(log=None):
    import torch

    import paper_2504_07042_amd as ax
    from paper_2504_07042_amd import meshgen

    out = {}

    def put(name, Y):
        torch.cuda.synchronize()
        out[name] = Y.detach().cpu().numpy().copy()

    def say(name):
        if log:
            print(f"[lds-poison] {name}", file=log, flush=True)

    tri = meshgen.jittered_hex(7, 5, 3, alpha=0.15, seed=11)       # 105 elements
    para, _ = meshgen.parallelepiped_hex(5, 5, 3, seed=4)             # 75 elements
    Vt = torch.from_numpy(tri.verts).cuda()
    Hp = ax.parallelepiped_factors(torch.from_numpy(para.verts).cuda())
    for N in range(1, 16):
        b = ax.Basis(N)
        for prec, dt in ((ax.AX_FP64, torch.float64), (ax.AX_FP32, torch.float32)):
            p = "fp64" if prec == ax.AX_FP64 else "fp32"
            for geom, V, E, tag in ((ax.AX_TRILINEAR, Vt, tri.E, "tri"), (ax.AX_PARALLELEPIPED, Hp, para.E, "para")):
                say(f"ax_local {tag} {p} N={N}")
                X = meshgen.random_nodal_device(E, N, nrhs=2, seed=N, dtype=dt)
                put(f"ax_local_{tag}_{p}_N{N}", ax.ax_local(X, V, b, geom, prec))
            if N in (3, 7, 8, 9, 12):
                say(f"stored {p} N={N}")
                G, _ = ax.geom_factors(Vt, b, prec)
                X = meshgen.random_nodal_device(tri.E, N, seed=N + 1, dtype=dt)
                put(f"stored_{p}_N{N}", ax.ax_local_precomputedG(X, G, b, prec))
                say(f"partial {p} N={N}")
                lam = ax.geom_lambda(Vt, b, prec)
                put(f"partial_{p}_N{N}", ax.ax_local_partial(X, Vt, lam, b, prec))
                say(f"helmholtz {p} N={N}")
                l0 = torch.full((tri.E, (N + 1) ** 3), 1.0, dtype=torch.float64, device="cuda")
                l1 = torch.full((tri.E, (N + 1) ** 3), 0.25, dtype=torch.float64, device="cuda")
                L23 = ax.helmholtz_factors(Vt, l0, l1, b, prec)
                put(f"helmholtz_{p}_N{N}", ax.ax_local_helmholtz(X, Vt, L23, b, prec))
                say(f"vector {p} N={N}")
                Xv = meshgen.random_nodal_device(tri.E, N, nrhs=3, seed=N + 2, dtype=dt)
                Xv = Xv.reshape(3, tri.E, -1).transpose(0, 1).contiguous()
                put(f"vector_{p}_N{N}", ax.ax_local_vector(Xv, Vt, b, ax.AX_TRILINEAR, prec))
    b7 = ax.Basis(7)
    for geom, V, E, tag in ((ax.AX_TRILINEAR, Vt, tri.E, "tri"), (ax.AX_PARALLELEPIPED, Hp, para.E, "para")):
        say(f"fp16 {tag} N=7")
        X = meshgen.random_nodal_device(E, 7, seed=3, dtype=torch.float32)
        put(f"fp16_{tag}_N7", ax.ax_local(X, V, b7, geom, ax.AX_FP16_ACC32))
    # batched: several meshes of uneven size and order in one plan, and the allocation-free call
    specs = [(3, (4, 3, 5)), (7, (3, 3, 3)), (5, (6, 2, 3)), (9, (2, 3, 2)), (7, (5, 4, 1)), (2, (3, 3, 3))]
    for prec, dt, p in ((ax.AX_FP64, torch.float64, "fp64"), (ax.AX_FP32, torch.float32, "fp32")):
        meshes, X, Y, Y2 = [], [], [], []
        for q, (N, dims) in enumerate(specs):
            m = meshgen.jittered_hex(*dims, alpha=0.12, seed=70 + q)
            meshes.append((torch.from_numpy(m.verts).cuda(), ax.Basis(N)))
            X.append(meshgen.random_nodal_device(m.E, N, nrhs=2, seed=q, dtype=dt))
            Y.append(torch.empty_like(X[-1]))
            Y2.append(torch.empty_like(X[-1]))
        say(f"batched {p}")
        plan = ax.BatchedAxLocal(meshes, X, Y, prec)
        plan.launch()
        for q in range(len(specs)):
            put(f"batched_{p}_{q}", Y[q])
        say(f"batched_noalloc {p}")
        ax.batched_noalloc(meshes, X, Y2, prec)
        for q in range(len(specs)):
            put(f"batched_noalloc_{p}_{q}", Y2[q])
    return out


if __name__ == "__main__":
    res = run_all(log=sys.stdout)
    np.savez(sys.argv[1], **res)
    print(f"[lds-poison] wrote {len(res)} cases", flush=True)
