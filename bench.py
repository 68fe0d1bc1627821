"""Benchmark: AxLocal throughput (GDOF/s) and roofline fraction on one MI355X.

Workload (one "step" = one application of the element-local Poisson operator with on-the-fly
trilinear geometric factors, FP64): N = 7 (8^3 GLL nodes per element), E = 32^3 = 32768
trilinear hexes of the unit cube with interior vertices jittered by +-15 % of h (seed 7),
X ~ U[-1, 1] (16.8 M local DOFs).  Inputs are resident in HBM before timing; four X/Y pairs
(1 GiB) rotate so that every step streams from HBM rather than the 256 MB Infinity Cache.

Prints ONE JSON line (rank 0).  Besides the headline, the default run adds: the measured HBM
bandwidth and arithmetic peaks of the device; the stored-factor baseline (the roofline the paper
raises), partial recomputation, Helmholtz, FP32, vector field and parallelepipeds on the same
size; the trilinear order sweep N in {3,5,7,9,11,15} at ~2^24 local nodes (FP64 and FP32;
on-the-fly, stored, partial); the FP64 and mixed-precision CG of the manufactured Poisson problem
with a Table 5-style line; the 64-mesh, 8-column batch (graph-replayed) with a sampled oracle
check; CG on the union of the batch (FP64 and FP32 reliable updates, one column); and the CPU
oracle timed on a bounded sample.  --no-extras keeps the headline only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
PEAK_FP64_TFS = 78.6        # MI355X FP64 vector (= FP64 matrix)
PEAK_FP32_TFS = 157.3
BASELINE_METRIC = "AxLocal GDOF/s + % roofline (N=7 trilinear FP64); mixed-prec CG speedup at 1e-10"


def flops_per_element(N, geom="tri", nrhs=1):
    """Per-element FLOPs: F_ax (Table 2, Poisson) per column plus F_geo (Table 3): trilinear
    72 N1 + 45 N1^2 + 80 N1^3, trilinear with partial recomputation 72 N1 + 45 N1^2 + 60 N1^3
    (Helmholtz with merged factors: plus the mass term, 2 N1^3), parallelepiped 7 N1^3, stored
    factors 0."""
    N1 = N + 1
    f_ax = 12 * N1**4 + 15 * N1**3
    f_geo = {"tri": 72 * N1 + 45 * N1**2 + 80 * N1**3, "partial": 72 * N1 + 45 * N1**2 + 60 * N1**3,
             "helm": 72 * N1 + 45 * N1**2 + 62 * N1**3, "para": 7 * N1**3, "stored": 0}[geom]
    return nrhs * f_ax, f_geo


def bytes_per_element(N, geom="tri", nrhs=1, fpsize=8):
    """Algorithmic HBM bytes per element: X read + Y write (nrhs columns) plus the geometry input
    (24 vertex words; plus N1^3 scale words with partial recomputation, 2 N1^3 merged factors
    for Helmholtz; 6 h words; or 6 N1^3 stored factors); D is cache-resident."""
    N1 = N + 1
    geo = {"tri": 24 * 8, "partial": 24 * 8 + N1**3 * fpsize, "helm": 24 * 8 + 2 * N1**3 * fpsize,
           "para": 6 * 8, "stored": 6 * N1**3 * fpsize}[geom]
    return 2 * nrhs * N1**3 * fpsize + geo


def measured_traffic(N, E, prec="fp64"):
    """HBM bytes per launch of the headline kernel from the calibrated FETCH_SIZE / WRITE_SIZE
    passes recorded in the package (measured_traffic.json), or None when the kernel sources have
    changed since those counters were taken or the workload differs."""
    import hashlib
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2504_07042_amd")
    try:
        with open(os.path.join(pkg, "measured_traffic.json")) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(pkg, "csrc", name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    wl = rec["workload"]
    if h.hexdigest() != rec["sha256"] or wl["N"] != N or wl["E"] != E or wl.get("precision", "fp64") != prec:
        return None
    return int(rec["bytes_per_launch"])


def time_steps(fn, steps, warmup, nbuf):
    """Warm up, then time `steps` calls (buffer index rotates) by wall clock between two device
    synchronisations, then run `steps` more calls with one event pair per call on torch's current
    stream (the stream every library call is enqueued on) for the per-launch kernel time.  The
    timed pass records no events: an event pair around every launch adds 4-6 us of stream gaps per
    step at N = 7 (measured: 78-79 us per step bare, 82-85 us with the events)."""
    import torch
    for s in range(warmup):
        fn(s % nbuf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        fn(s % nbuf)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for s in range(steps):
        ev[s][0].record()
        fn(s % nbuf)
        ev[s][1].record()
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
    return wall, per


def measure_peaks(ax, dev):
    """Sustained rates of this device, for the time-based roofline of Sec. 3.4 (which divides by
    measured bandwidth): the library's HBM copy probe over a 1 GiB footprint (two rotating pairs of
    512 MiB buffers; one read and one write per byte) and its arithmetic probes (FP64 / FP32 fused
    multiply-add on the vector ALU, FP32 unpacked as the library is built; 16x16x4 matrix-core
    loops; FP64 vector and matrix loops issued together).  Medians of 10 timed launches."""
    import torch
    nb = 512 * 2**20
    bufs = [(torch.ones(nb, dtype=torch.uint8, device=dev), torch.empty(nb, dtype=torch.uint8, device=dev))
            for _ in range(2)]
    _, per = time_steps(lambda q: ax.probe_copy(bufs[q][0], bufs[q][1]), 20, 10, 2)
    del bufs
    torch.cuda.empty_cache()
    bmeas = 2 * nb / float(np.median(per)) / 1e9
    out = {"hbm_copy_GBs": round(bmeas, 1), "hbm_copy_frac_of_8000": round(bmeas / PEAK_HBM_GBS, 3),
           "copy_footprint_bytes": 2 * nb}
    times = {}
    for name, kind, iters in (("fp64_valu_fma", ax.AX_PROBE_FMA_F64, 1000),
                              ("fp64_mfma_16x16x4", ax.AX_PROBE_MFMA_F64, 1000),
                              ("fp64_valu_and_mfma_together", ax.AX_PROBE_MIX_F64, 1000),
                              ("fp32_valu_fma_unpacked", ax.AX_PROBE_FMA_F32, 1000),
                              ("fp32_mfma_16x16x4", ax.AX_PROBE_MFMA_F32, 1000)):
        buf, fl = ax.probe_compute(kind, iters)
        _, per = time_steps(lambda q: ax.probe_compute(kind, iters, out=buf), 10, 3, 1)
        t = float(np.median(per))
        times[name] = t
        out[name + "_TFs"] = round(fl / t / 1e12, 2)
    # the mixed probe runs the FP64 vector loop and the matrix loop of the two probes before it in
    # the same waves: time / (sum of the separate times) near 1 means no overlap, near
    # max / sum that the two units run concurrently
    tv, tm, tb = times["fp64_valu_fma"], times["fp64_mfma_16x16x4"], times["fp64_valu_and_mfma_together"]
    out["fp64_together_time_over_sum"] = round(tb / (tv + tm), 3)
    out["fp64_together_time_over_max"] = round(tb / max(tv, tm), 3)
    return out


def cpu_baseline(mesh, N, X, budget_s=10.0):
    """The oracle (plain FP64 loops, OpenMP over elements): stored factors from the vertices
    (Eq. 7) then AxLocal (Algorithm 1), on a bounded sample of the same mesh, repeated until
    about `budget_s` seconds of CPU time have elapsed."""
    import oracle
    xi, w, D = oracle.gll(N)
    nsamp = min(mesh.E, 4096)
    V = np.ascontiguousarray(mesh.verts[:nsamp])
    Xs = np.ascontiguousarray(X[:, :nsamp])
    reps = 0
    t0 = time.perf_counter()
    while True:
        G, _, _ = oracle.geom_factors(V, N, xi, w)
        oracle.ax_local(D, G, Xs)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    dofs = reps * nsamp * (N + 1) ** 3 * X.shape[0]
    cores = oracle.num_threads()
    # the same on one core, on a smaller sample
    n1 = min(nsamp, 256)
    oracle.set_num_threads(1)
    reps1, t1 = 0, time.perf_counter()
    while True:
        G, _, _ = oracle.geom_factors(V[:n1], N, xi, w)
        oracle.ax_local(D, G, Xs[:, :n1])
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= budget_s / 4:
            break
    oracle.set_num_threads(cores)
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"value": dofs / el / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": f"{nsamp} of {mesh.E} elements (first {nsamp}), N={N}, nrhs={X.shape[0]}, "
                      f"geometric factors + AxLocal, {reps} repetitions in {el:.1f} s",
            "single_core_GDOFs": reps1 * n1 * (N + 1) ** 3 * X.shape[0] / el1 / 1e9,
            "os_cpu_count": os.cpu_count(), "affinity_cpus": aff}


def cg_solves(ax, meshgen, dev, N=7, grid=(32, 32, 32), rtol=1e-10, check_with_oracle=True, fp16=False):
    """-Lap u = f on the unit cube (homogeneous Dirichlet), N = 7, 32^3 trilinear hexes with
    +-10 % jitter (seed 4), f from u = sin(pi x) sin(pi y) sin(pi z).  Time to a true relative
    residual of 1e-10: plain FP64 CG against mixed precision with an FP32 inner AxLocal (reliable
    updates, and restarted refinement) and an FP16 (matrix-core) inner AxLocal (restarted); and
    the Jacobi-preconditioned solves (FP64, FP32 reliable updates)."""
    import torch
    m = meshgen.jittered_hex(*grid, alpha=0.10, seed=4)
    l2g, ng, mask = meshgen.global_numbering(*grid, N)
    b = ax.Basis(N)
    gs = ax.GatherScatter(l2g, ng, mask)
    V = torch.from_numpy(m.verts).to(dev)
    prob = ax.Problem(V, b, gs)
    # right-hand side b = mask o Q^T (w det J o f) (lumped mass) at the physical nodes
    XYZ = ax.node_coords(V, b)
    _, gwj = ax.geom_factors(V, b, want_G=False, want_gwj=True)
    f = 3 * np.pi**2 * torch.sin(np.pi * XYZ[:, 0]) * torch.sin(np.pi * XYZ[:, 1]) * torch.sin(np.pi * XYZ[:, 2])
    rhs = gs.apply((gwj * f).reshape(1, -1).contiguous(), ax.GS_QT)
    torch.cuda.synchronize()
    res = {"workload": f"Poisson N={N} E={grid[0]}x{grid[1]}x{grid[2]} jitter 10% seed 4, global DOFs {ng}",
           "rtol": rtol}
    runs = [("fp64", dict(inner_prec=ax.AX_FP64)),
            ("mixed_fp32_reliable", dict(inner_prec=ax.AX_FP32, inner_rtol=0.1, refine=ax.AX_REFINE_RELIABLE)),
            ("mixed_fp32_restart", dict(inner_prec=ax.AX_FP32, inner_rtol=1e-5)),
            # Jacobi-preconditioned CG (a Table 5-style solve; the paper does not name the
            # preconditioner), FP64 and mixed
            ("jacobi_fp64", dict(inner_prec=ax.AX_FP64, precond=ax.AX_PRECOND_JACOBI)),
            ("jacobi_mixed_fp32_reliable", dict(inner_prec=ax.AX_FP32, inner_rtol=0.1, refine=ax.AX_REFINE_RELIABLE,
                                                precond=ax.AX_PRECOND_JACOBI))]
    if fp16:
        # half-precision inner operator (N = 7 only); slower than plain FP64 on MI355X
        runs.append(("mixed_fp16_restart", dict(inner_prec=ax.AX_FP16_ACC32, inner_rtol=1e-2)))
    # per-launch AxLocal time on this mesh in each precision (for the AxLocal share of a solve)
    t_ax = {}
    xl = meshgen.random_nodal_device(m.E, N, 1, seed=9, device=dev)
    for pname, prec, T in (("fp64", ax.AX_FP64, torch.float64), ("fp32", ax.AX_FP32, torch.float32),
                           ("fp16", ax.AX_FP16_ACC32, torch.float32)):
        xx = xl.to(T)
        yy = torch.empty_like(xx)
        _, per = time_steps(lambda q: ax.ax_local(xx, V, b, ax.AX_TRILINEAR, prec, out=yy), 50, 20, 1)
        t_ax[pname] = float(np.median(per))
    del xl, xx, yy
    f_ax, _ = flops_per_element(N, "tri")
    sols = {}
    for name, kw in runs:
        x, rep = ax.cg_solve(prob, rhs, rtol=rtol, max_it=40000, max_outer=60, **kw)
        ent = {k: (round(v, 4) if isinstance(v, float) and k == "seconds" else v) for k, v in rep.items()}
        its, sec = rep["iterations"], rep["seconds"]
        inner = {ax.AX_FP64: "fp64", ax.AX_FP32: "fp32", ax.AX_FP16_ACC32: "fp16"}[kw["inner_prec"]]
        n_fp64_apps = 0 if inner == "fp64" else rep["outer_it"] + 1
        if sec > 0 and its > 0:
            # Table 5 style: GDOFS = global DOFs x iterations / time; GFLOPS counts per iteration
            # the AxLocal flops of Table 2 (E F_ax) and 10 flops per global DOF of CG vector work
            ent["table5"] = {"GDOFS": round(ng * its / sec / 1e9, 3),
                             "GFLOPS": round((m.E * f_ax + 10 * ng) * its / sec / 1e9, 1),
                             "axlocal_share_est": round((its * t_ax[inner] + n_fp64_apps * t_ax["fp64"]) / sec, 3),
                             "iterations": its}
        res[name] = ent
        sols[name] = x
    res["axlocal_us_per_launch"] = {k: round(v * 1e6, 1) for k, v in t_ax.items()}
    t64 = res["fp64"]["seconds"]
    for name, _ in runs[1:]:
        res[name]["speedup_vs_fp64"] = round(t64 / res[name]["seconds"], 3) if res[name]["seconds"] > 0 else None
    tj = res["jacobi_fp64"]["seconds"]
    res["jacobi_mixed_fp32_reliable"]["speedup_vs_jacobi_fp64"] = (
        round(tj / res["jacobi_mixed_fp32_reliable"]["seconds"], 3) if res["jacobi_mixed_fp32_reliable"]["seconds"] > 0
        else None)
    ug = torch.zeros(ng, dtype=torch.float64, device=dev)
    u = torch.sin(np.pi * XYZ[:, 0]) * torch.sin(np.pi * XYZ[:, 1]) * torch.sin(np.pi * XYZ[:, 2])
    ug[gs.l2g.long()] = u.reshape(-1)
    res["max_nodal_error_fp64"] = float((sols["fp64"][0] - ug).abs().max())
    for name in sols:
        if "table5" in res[name]:
            res[name]["table5"]["max_nodal_error"] = float((sols[name][0] - ug).abs().max())
    if check_with_oracle:
        import oracle
        xi, w, D = oracle.gll(N)
        G, _, _ = oracle.geom_factors(m.verts, N, xi, w)
        bh = rhs[0].cpu().numpy()
        for name in sols:
            xh = sols[name][0].cpu().numpy()
            r = bh - oracle.apply_A(N, D, G, l2g, ng, mask, xh)
            res[name]["oracle_rel_res"] = float(np.linalg.norm(r) / np.linalg.norm(bh))
        del G
    return res


def roofline_gdofs(N, geom, fpsize=8, peak_tf=PEAK_FP64_TFS, peak_gbs=PEAK_HBM_GBS, nrhs=1):
    """Time-based roofline (Sec. 3.4) in local DOFs per second (nrhs columns count nrhs DOFs
    per node): max(T_cmp, T_mem) per element."""
    f_ax, f_geo = flops_per_element(N, geom, nrhs)
    t_cmp = (f_ax + f_geo) / (peak_tf * 1e12)
    t_mem = bytes_per_element(N, geom, nrhs=nrhs, fpsize=fpsize) / (peak_gbs * 1e9)
    return nrhs * (N + 1) ** 3 / max(t_cmp, t_mem) / 1e9, ("alu" if t_cmp >= t_mem else "hbm")


def order_sweep(ax, meshgen, dev, orders=(3, 5, 7, 9, 11, 15), steps=20, warmup=10, nbuf=4, peaks=None):
    """Trilinear order sweep at E (N+1)^3 ~ 2^24 local nodes, +-15 % jitter, seed N: on-the-fly,
    stored factors and partial recomputation, FP64 and FP32, each against its time-based roofline
    (datasheet peaks, and the measured ones when `peaks` is given).  nbuf X/Y pairs rotate (1 GiB
    in FP64, 512 MiB in FP32) so every launch streams from HBM, not the 256 MB Infinity Cache."""
    import torch
    rows = []
    bmeas = peaks["hbm_copy_GBs"] if peaks else None
    for N in orders:
        grid = meshgen.grid_for_nodes(N)
        m = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
        b = ax.Basis(N)
        V = torch.from_numpy(m.verts).to(dev)
        X64 = torch.from_numpy(meshgen.random_nodal(m.E, N, seed=N)).to(dev)
        row = {"N": N, "E": m.E, "grid": list(grid), "local_dofs": m.E * (N + 1) ** 3}
        for pname, prec, T in (("fp64", ax.AX_FP64, torch.float64), ("fp32", ax.AX_FP32, torch.float32)):
            X = [X64.to(T) for _ in range(nbuf)]
            Y = [torch.empty_like(x) for x in X]
            fpsize = 8 if T == torch.float64 else 4
            peak = PEAK_FP64_TFS if T == torch.float64 else PEAK_FP32_TFS
            pmeas = None
            if peaks:
                pmeas = peaks["fp64_valu_fma_TFs"] if T == torch.float64 else peaks["fp32_valu_fma_unpacked_TFs"]
            res = {}
            for var in ("tri", "stored", "partial"):
                if var == "tri":
                    fn = lambda q: ax.ax_local(X[q], V, b, ax.AX_TRILINEAR, prec, out=Y[q])
                elif var == "stored":
                    G, _ = ax.geom_factors(V, b, prec)
                    fn = lambda q: ax.ax_local_precomputedG(X[q], G, b, prec, out=Y[q])
                else:
                    lam = ax.geom_lambda(V, b, prec)
                    fn = lambda q: ax.ax_local_partial(X[q], V, lam, b, prec, out=Y[q])
                _, per = time_steps(fn, steps, warmup, nbuf)
                g = row["local_dofs"] / float(np.median(per)) / 1e9
                r, bound = roofline_gdofs(N, var, fpsize, peak)
                ent = {"GDOFs": round(g, 1), "us": round(float(np.median(per)) * 1e6, 1), "R_GDOFs": round(r, 1),
                       "bound": bound, "frac_of_R": round(g / r, 3)}
                if peaks:
                    rm, bm = roofline_gdofs(N, var, fpsize, pmeas, bmeas)
                    ent.update({"R_measured_GDOFs": round(rm, 1), "bound_measured": bm, "frac_of_R_measured": round(g / rm, 3)})
                res[var] = ent
                fn = None
                G = lam = None
                torch.cuda.empty_cache()
            res["speedup_on_the_fly_vs_stored"] = round(res["tri"]["GDOFs"] / res["stored"]["GDOFs"], 2)
            row[pname] = res
            del X, Y
        rows.append(row)
        print(f"sweep N={N}: " + json.dumps({k: row[k] for k in ("fp64", "fp32")}), file=sys.stderr, flush=True)
        del X64, V
        torch.cuda.empty_cache()
    return rows


def element_sweep(ax, meshgen, dev, N=7, steps=20, warmup=20):
    """Trilinear FP64 AxLocal at N = 7 for E = 2^15 ... 2^20 elements (one X/Y pair, +-15 %
    jitter, seed N): the plateau of the throughput with the problem size, from inside the 256 MB
    Infinity Cache (X and Y of E = 2^15 take 256 MiB) to far outside it."""
    import torch
    rows = []
    b = ax.Basis(N)
    for grid in ((32, 32, 32), (64, 32, 32), (64, 64, 32), (64, 64, 64), (128, 64, 64), (128, 128, 64)):
        m = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
        V = torch.from_numpy(m.verts).to(dev)
        del m
        X = meshgen.random_nodal_device(V.shape[0], N, seed=N, device=dev)
        Y = torch.empty_like(X)
        # warm up for a fixed time (the clocks need about 0.2 s of continuous launches to ramp)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.3:
            for _ in range(10):
                ax.ax_local(X, V, b, ax.AX_TRILINEAR, ax.AX_FP64, out=Y)
            torch.cuda.synchronize()
        _, per = time_steps(lambda q: ax.ax_local(X, V, b, ax.AX_TRILINEAR, ax.AX_FP64, out=Y), steps, warmup, 1)
        dofs = V.shape[0] * (N + 1) ** 3
        rows.append({"E": V.shape[0], "grid": list(grid), "local_dofs": dofs,
                     "x_plus_y_MiB": round(2 * dofs * 8 / 2**20), "GDOFs": round(dofs / per.mean() / 1e9, 1),
                     "us_per_launch": round(per.mean() * 1e6, 1)})
        del X, Y, V
        torch.cuda.empty_cache()
    return rows


def batched_run(ax, meshgen, dev, nrhs=8, steps=5, warmup=2, check_with_oracle=True):
    """64 independent trilinear meshes (E ~ U[512, 32768] rounded to a near-cubic grid, N drawn
    from {3, 5, 7, 9}, seed 1, +-10 % jitter) with 8 columns each: one persistent launch (replayed
    from a HIP graph) against one ax_local launch per mesh, FP64 and FP32."""
    import torch
    specs = meshgen.batch_specs(64, 512, 32768, (3, 5, 7, 9), seed=1)
    meshes, verts_h = [], []
    for sp in specs:
        m = meshgen.jittered_hex(sp.nx, sp.ny, sp.nz, alpha=0.10, seed=sp.seed)
        verts_h.append(m.verts)
        meshes.append((torch.from_numpy(m.verts).to(dev), ax.Basis(sp.N)))
    dofs = sum(v.shape[0] * (sp.N + 1) ** 3 for v, sp in zip(verts_h, specs)) * nrhs
    res = {"workload": f"64 meshes, N in {{3,5,7,9}}, E in [{min(v.shape[0] for v in verts_h)}, "
                       f"{max(v.shape[0] for v in verts_h)}], {nrhs} columns, {dofs} local DOFs", "local_dofs": dofs}
    for pname, prec, T in (("fp64", ax.AX_FP64, torch.float64), ("fp32", ax.AX_FP32, torch.float32)):
        X = [meshgen.random_nodal_device(v.shape[0], sp.N, nrhs, seed=q, device=dev, dtype=T)
             for q, (v, sp) in enumerate(zip(verts_h, specs))]
        Y = [torch.empty_like(x) for x in X]
        bat = ax.BatchedAxLocal(meshes, X, Y, prec)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            bat.launch(stream=s)
            with torch.cuda.graph(g, stream=s):
                bat.launch(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        wall_b, per_b = time_steps(lambda q: g.replay(), steps, warmup, 1)
        Yb = [y.clone() for y in Y] if check_with_oracle else None

        def per_mesh(q):
            for (v, b), x, y in zip(meshes, X, Y):
                ax.ax_local(x, v, b, ax.AX_TRILINEAR, prec, out=y)

        wall_l, per_l = time_steps(per_mesh, steps, warmup, 1)
        from paper_2504_07042_amd import item_shape_of
        shapes = {f"N={N1 - 1}": item_shape_of(N1, bat.plan.order_variant[N1], prec)
                  for N1 in range(2, 11) if bat.plan.order_count[N1] > 0}
        res[pname] = {"batched_graph_GDOFs": round(dofs / per_b.mean() / 1e9, 1),
                      "per_mesh_launches_GDOFs": round(dofs / per_l.mean() / 1e9, 1),
                      "batched_ms": round(per_b.mean() * 1e3, 3), "per_mesh_ms": round(per_l.mean() * 1e3, 3),
                      "work_group_shapes": shapes}
        if Yb is not None:
            import oracle
            worst = 0.0
            rng = np.random.default_rng(0)
            for q in rng.choice(len(specs), 4, replace=False):
                N = specs[q].N
                sel = np.sort(rng.choice(verts_h[q].shape[0], 16, replace=False))
                xi, w, D = oracle.gll(N)
                G, _, _ = oracle.geom_factors(verts_h[q][sel], N, xi, w)
                xs = X[q][:, sel].cpu().numpy().astype(np.float64)
                yr = oracle.ax_local(D, G, xs)
                env = oracle.ax_envelope(D, G, xs)
                d = np.abs(Yb[q][:, sel].cpu().numpy().astype(np.float64) - yr) / np.maximum(env, 1e-300)
                worst = max(worst, float(d.max()))
            res[pname]["oracle_sampled_max_err_over_env"] = worst
        del X, Y, bat, g
        torch.cuda.empty_cache()
    return res


def batched_cg(ax, meshgen, dev, rtol=1e-10, nrhs=1, restart_leg=False):
    """CG on the block-diagonal union of the 64 batched meshes (same specs as batched_run), every
    AxLocal application of a step in one persistent launch: plain FP64 against mixed precision
    (FP32 inner AxLocal, reliable updates and restarted refinement), time to a true relative
    residual of 1e-10.  b ~ U[-1, 1] per global node, zero on each box boundary."""
    import torch
    specs = meshgen.batch_specs(64, 512, 32768, (3, 5, 7, 9), seed=1)
    meshes, parts = [], []
    for sp in specs:
        m = meshgen.jittered_hex(sp.nx, sp.ny, sp.nz, alpha=0.10, seed=sp.seed)
        meshes.append((torch.from_numpy(m.verts).to(dev), ax.Basis(sp.N)))
        parts.append(meshgen.global_numbering(sp.nx, sp.ny, sp.nz, sp.N))
    l2g, ng, mask, _, _ = meshgen.concat_numbering(parts)
    del parts
    gs = ax.GatherScatter(l2g, ng, mask)
    b = meshgen.random_global_device(ng, mask, nrhs, seed=5, device=dev)
    res = {"workload": f"union of the 64 batched meshes, {l2g.size} local / {ng} global DOFs, {nrhs} column(s), "
                       f"b ~ U[-1,1]", "rtol": rtol}
    del l2g
    runs = [("fp64", dict(inner_prec=ax.AX_FP64)),
            ("mixed_fp32_reliable", dict(inner_prec=ax.AX_FP32, inner_rtol=0.1, refine=ax.AX_REFINE_RELIABLE))]
    if restart_leg:
        runs.append(("mixed_fp32_restart", dict(inner_prec=ax.AX_FP32, inner_rtol=1e-5)))
    res["legs"] = [r[0] for r in runs]
    for name, kw in runs:
        x, rep = ax.cg_solve_batched(meshes, gs, b, rtol=rtol, max_it=20000, max_outer=80, **kw)
        res[name] = {k: (round(v, 4) if isinstance(v, float) and k == "seconds" else v) for k, v in rep.items()}
        print(f"batched cg {name}: {res[name]}", file=sys.stderr, flush=True)
        del x
    t64 = res["fp64"]["seconds"]
    for name, _ in runs[1:]:
        res[name]["speedup_vs_fp64"] = round(t64 / res[name]["seconds"], 3) if res[name]["seconds"] > 0 else None
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--N", type=int, default=7)
    ap.add_argument("--prec", choices=("fp64", "fp32"), default="fp64",
                    help="arithmetic of the headline leg (fp32 only with --no-extras; for profiling the FP32 kernel)")
    ap.add_argument("--grid", type=int, nargs=3, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="only the headline kernel")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 128 MiB device copy (counter calibration)")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG / mixed-precision solves")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched workload: 64 meshes, E~U[512,32768], N in {3,5,7,9}, 8 columns")
    ap.add_argument("--no-batched-cg", action="store_true",
                    help="skip CG (FP64 vs FP32 reliable updates) on the union of the 64 batched meshes (minutes)")
    ap.add_argument("--batched-cg-restart", action="store_true",
                    help="add the restarted-refinement leg to the batched CG")
    ap.add_argument("--esweep", action="store_true",
                    help="also run the element-count sweep E = 2^15..2^20 at N = 7 (trilinear FP64)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the order sweep N in {3,5,7,9,11,15} at ~2^24 local nodes")
    ap.add_argument("--no-peaks", action="store_true", help="skip the bandwidth and arithmetic probes")
    ap.add_argument("--only-cg", action="store_true",
                    help="headline and the single-mesh CG legs only (for profiling the solver)")
    ap.add_argument("--fp16-cg", action="store_true",
                    help="add the CG leg with the half-precision (matrix-core) inner operator")
    args = ap.parse_args(argv)

    if args.prec != "fp64" and not args.no_extras:
        print("--prec fp32 profiles the FP32 headline kernel only: add --no-extras", file=sys.stderr)
        return 2
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only; run with --gpus 1 "
              "(the element-parallel operator would shard by element slabs, one per GPU)", file=sys.stderr)
        return 2

    import torch
    import paper_2504_07042_amd as ax
    from paper_2504_07042_amd import autotune
    from paper_2504_07042_amd import meshgen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    ax.lib()
    dev = torch.device("cuda:0")
    N = args.N
    N1 = N + 1
    grid = tuple(args.grid) if args.grid else meshgen.grid_for_nodes(N)
    mesh = meshgen.jittered_hex(*grid, alpha=0.15, seed=N)
    E = mesh.E
    NP = N1**3
    b = ax.Basis(N)
    NBUF = 4
    X_host = meshgen.random_nodal(E, N, nrhs=1, seed=N)
    f64 = args.prec == "fp64"
    hprec = ax.AX_FP64 if f64 else ax.AX_FP32
    Xs = [torch.from_numpy(X_host).to(dev).to(torch.float64 if f64 else torch.float32) for _ in range(NBUF)]
    Ys = [torch.empty_like(Xs[0]) for _ in range(NBUF)]
    V = torch.from_numpy(mesh.verts).to(dev)
    torch.cuda.synchronize()
    PEAK = PEAK_FP64_TFS if f64 else PEAK_FP32_TFS

    def step(q):
        ax.ax_local(Xs[q], V, b, ax.AX_TRILINEAR, hprec, out=Ys[q])

    # the machine probes (part of the report) run first: a second or two of full load that also
    # brings the clocks to their loaded state before the headline's own warm-up steps
    peaks = None if args.no_peaks else measure_peaks(ax, dev)
    wall, per = time_steps(step, args.steps, args.warmup, NBUF)
    t_kernel = float(per.mean())
    dofs = E * NP
    gdofs = dofs * args.steps / wall / 1e9
    f_ax, f_geo = flops_per_element(N, "tri")
    by = bytes_per_element(N, "tri", fpsize=8 if f64 else 4)
    achieved_tf = (f_ax + f_geo) * E / t_kernel / 1e12
    achieved_gbs = by * E / t_kernel / 1e9
    # time-based roofline (Sec. 3.4): T_cmp = (F_ax + F_geo) / P, T_mem = M / B
    t_cmp = (f_ax + f_geo) * E / (PEAK * 1e12)
    t_mem = by * E / (PEAK_HBM_GBS * 1e9)
    compute_bound = t_cmp >= t_mem
    roofline = {
        "bound": "alu" if compute_bound else "hbm",
        "achieved": round(achieved_tf if compute_bound else achieved_gbs, 3),
        "peak": PEAK if compute_bound else PEAK_HBM_GBS,
        "unit": "TFLOP/s" if compute_bound else "GB/s",
        "frac": round((achieved_tf / PEAK) if compute_bound else (achieved_gbs / PEAK_HBM_GBS), 4),
        "traffic": measured_traffic(N, E, args.prec),
        "kernel": f"ax_local_kernel<N1={N1}, trilinear, {'double' if f64 else 'float'}>",
        "per_launch": {"elements": E, "flops_per_element": f_ax + f_geo, "bytes_per_element": by,
                       "avg_launch_ms": round(t_kernel * 1e3, 4)},
        "hbm_GBs_achieved": round(achieved_gbs, 1),
        "R_eff_GDOFs": round(dofs / max(t_cmp, t_mem) / 1e9, 1),
        "pct_of_R_eff": round(max(t_cmp, t_mem) / t_kernel, 4),
        "time_base": "mean HIP-event time per launch on the launch stream (value uses the wall time of "
                     "the timed steps)",
        "frac_wall_clock": round((f_ax + f_geo) * E / (wall / args.steps) / 1e12 / PEAK, 4)
        if compute_bound else round(by * E / (wall / args.steps) / 1e9 / PEAK_HBM_GBS, 4),
    }

    if peaks is not None:
        pm = peaks["fp64_valu_fma_TFs"] if f64 else peaks["fp32_valu_fma_unpacked_TFs"]
        roofline["peak_measured"] = pm if compute_bound else peaks["hbm_copy_GBs"]
        roofline["frac_of_measured_peak"] = round(roofline["achieved"] / roofline["peak_measured"], 4)
        t_cmp_m = (f_ax + f_geo) * E / (pm * 1e12)
        t_mem_m = by * E / (peaks["hbm_copy_GBs"] * 1e9)
        roofline["R_eff_measured_GDOFs"] = round(dofs / max(t_cmp_m, t_mem_m) / 1e9, 1)
        roofline["pct_of_R_eff_measured"] = round(max(t_cmp_m, t_mem_m) / t_kernel, 4)

    out = {
        "metric": BASELINE_METRIC,
        "value": round(gdofs, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"AxLocal trilinear N={N} E={grid[0]}x{grid[1]}x{grid[2]}={E} jitter 15% seed {N}",
                   "N": N, "E": E, "local_dofs": dofs, "nrhs": 1, "geometry": "trilinear",
                   "precision": args.prec, "tuning_cache": autotune.cache_status(),
                   "launch": {k: v for k, v in autotune.tune_get(N, ax.AX_TUNE_TRILINEAR, hprec).items()
                              if k in ("kernel_used", "elems_per_group", "block", "waves", "grid_mult")}},
        "roofline": roofline,
    }

    if args.only_cg:
        args.no_extras = True
    if not args.no_extras:
        extras = {}
        # stored-factor baseline on the same mesh: the roofline the paper raises
        G, _ = ax.geom_factors(V, b, ax.AX_FP64)

        def step_g(q):
            ax.ax_local_precomputedG(Xs[q], G, b, ax.AX_FP64, out=Ys[q])

        wall_g, per_g = time_steps(step_g, args.steps, args.warmup, NBUF)
        byg = bytes_per_element(N, "stored")
        extras["stored_G_fp64"] = {"GDOFs": round(dofs * args.steps / wall_g / 1e9, 3),
                                   "hbm_GBs": round(byg * E / per_g.mean() / 1e9, 1),
                                   "R_orig_GDOFs": round(dofs / (byg * E / (PEAK_HBM_GBS * 1e9)) / 1e9, 1)}
        extras["speedup_on_the_fly_vs_stored"] = round(wall_g / wall, 3)
        del G
        # partial recomputation (Sec. 4.2.2): the per-node scale read from memory
        lam = ax.geom_lambda(V, b, ax.AX_FP64)

        def step_p(q):
            ax.ax_local_partial(Xs[q], V, lam, b, ax.AX_FP64, out=Ys[q])

        wall_p, per_p = time_steps(step_p, args.steps, args.warmup, NBUF)
        fa_p, fg_p = flops_per_element(N, "partial")
        byp = bytes_per_element(N, "partial")
        r_p, bound_p = roofline_gdofs(N, "partial")
        extras["partial_recompute_fp64"] = {
            "GDOFs": round(dofs * args.steps / wall_p / 1e9, 3),
            "TFLOPs": round((fa_p + fg_p) * E / per_p.mean() / 1e12, 3),
            "hbm_GBs": round(byp * E / per_p.mean() / 1e9, 1),
            "R_eff_GDOFs": round(r_p, 1), "bound": bound_p,
            "pct_of_R_eff": round(dofs / per_p.mean() / 1e9 / r_p, 4),
            "vs_full_recompute": round(wall / wall_p, 3)}
        del lam
        # Helmholtz operator with merged scalar factors (Eq. 3, Sec. 4.2.1), seeded coefficient fields
        rng = np.random.default_rng(11)
        lam0 = torch.from_numpy(rng.uniform(0.5, 2.0, (E, NP))).to(dev)
        lam1 = torch.from_numpy(rng.uniform(0.0, 3.0, (E, NP))).to(dev)
        L23 = ax.helmholtz_factors(V, lam0, lam1, b, ax.AX_FP64)
        del lam0, lam1

        def step_h(q):
            ax.ax_local_helmholtz(Xs[q], V, L23, b, ax.AX_FP64, out=Ys[q])

        wall_h, per_h = time_steps(step_h, args.steps, args.warmup, NBUF)
        fa_h, fg_h = flops_per_element(N, "helm")
        byh = bytes_per_element(N, "helm")
        r_h, bound_h = roofline_gdofs(N, "helm")
        extras["helmholtz_merged_fp64"] = {
            "GDOFs": round(dofs * args.steps / wall_h / 1e9, 3),
            "TFLOPs": round((fa_h + fg_h) * E / per_h.mean() / 1e12, 3),
            "hbm_GBs": round(byh * E / per_h.mean() / 1e9, 1),
            "R_eff_GDOFs": round(r_h, 1), "bound": bound_h,
            "pct_of_R_eff": round(dofs / per_h.mean() / 1e9 / r_h, 4)}
        del L23
        # FP32 on-the-fly on the same mesh
        X32 = [x.float() for x in Xs]
        Y32 = [y.float() for y in Ys]

        def step32(q):
            ax.ax_local(X32[q], V, b, ax.AX_TRILINEAR, ax.AX_FP32, out=Y32[q])

        wall32, _ = time_steps(step32, args.steps, args.warmup, NBUF)
        extras["trilinear_fp32_GDOFs"] = round(dofs * args.steps / wall32 / 1e9, 3)
        del X32, Y32
        # vector field (n_col = 3, Sec. 4.1): the three components of an element contiguous
        # ([E][3][N1^3]) and sharing the recomputed factors; two rotating X/Y pairs (1.5 GiB)
        X3 = [meshgen.random_nodal_device(E, N, nrhs=3, seed=N + 3 + q, device=dev).reshape(E, 3, NP)
              for q in range(2)]
        Y3 = [torch.empty_like(x) for x in X3]
        wall3, per3 = time_steps(lambda q: ax.ax_local_vector(X3[q], V, b, ax.AX_TRILINEAR, ax.AX_FP64, out=Y3[q]),
                                 max(20, args.steps // 4), max(20, args.warmup // 4), 2)
        fa3, fg3 = flops_per_element(N, "tri", nrhs=3)
        r3, bound3 = roofline_gdofs(N, "tri", nrhs=3)
        extras["vector_field_ncol3_fp64"] = {
            "layout": "[E][3][N1^3] (ax_local_vector)",
            "GDOFs": round(3 * dofs / per3.mean() / 1e9, 3),
            "TFLOPs": round((fa3 + fg3) * E / per3.mean() / 1e12, 3),
            "hbm_GBs": round(bytes_per_element(N, "tri", nrhs=3) * E / per3.mean() / 1e9, 1),
            "R_eff_GDOFs": round(r3, 1), "bound": bound3,
            "pct_of_R_eff": round(3 * dofs / per3.mean() / 1e9 / r3, 4)}
        del X3, Y3
        # parallelepiped elements (32^3 sheared cube, N = 7)
        pm, _ = meshgen.parallelepiped_hex(*grid, seed=2)
        h = ax.parallelepiped_factors(torch.from_numpy(pm.verts).to(dev))

        def step_p(q):
            ax.ax_local(Xs[q], h, b, ax.AX_PARALLELEPIPED, ax.AX_FP64, out=Ys[q])

        wall_p, per_p = time_steps(step_p, args.steps, args.warmup, NBUF)
        byp = bytes_per_element(N, "para")
        extras["parallelepiped_fp64"] = {"GDOFs": round(dofs * args.steps / wall_p / 1e9, 3),
                                         "hbm_GBs": round(byp * E / per_p.mean() / 1e9, 1)}
        out["extras"] = extras

    if peaks:
        out["measured_peaks"] = peaks
    if not args.no_extras and not args.no_sweep:
        out["order_sweep"] = order_sweep(ax, meshgen, dev, steps=20, warmup=10, peaks=peaks)

    if (args.only_cg or not args.no_extras) and not args.no_cg:
        out["cg"] = cg_solves(ax, meshgen, dev, check_with_oracle=not args.no_cpu, fp16=args.fp16_cg)

    if not args.no_extras and not args.no_batched:
        out["batched"] = batched_run(ax, meshgen, dev, steps=10, warmup=3, check_with_oracle=not args.no_cpu)
    if not args.no_extras and not args.no_batched_cg:
        out["batched_cg"] = batched_cg(ax, meshgen, dev, restart_leg=args.batched_cg_restart)
    if args.esweep:
        out["element_sweep"] = element_sweep(ax, meshgen, dev)

    if args.calib:
        a = torch.empty(16 * 2**20, dtype=torch.float64, device=dev).uniform_()
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes_each_way"] = a.numel() * 8

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, N, X_host)

    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
