"""Benchmark of the stencil-scaling hot path on one MI355X.

One step = one application of the scaled-stencil operator (FP64) to one
synthetic field on the unit macro tetrahedron at level 8 (2,731,135
unknowns, lognormal k with sigma = 1, correlation length 0.1, seed 1).
`value` is that apply's throughput in GDoF/s (unknowns per second).  The same
run also reports, as context, the FP32 apply, the nodal-integration kernel,
the HBM-resident 48-tet level-8 working set, multigrid time to a 1e-8
relative residual (FP64 and FP32-in-FP64), the roofline of the dominant
kernel, and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scaled-stencil matvec GDoF/s + %HBM peak; V-cycle time to 1e-8 rel. residual"
HBM_PEAK_GBS = 8000.0
BYTES_PER_DOF = {"f64": 24, "f32": 12}   # read u and k, write y (perfect neighbour reuse)
PROFILE = os.path.join(ROOT, "profiles", "traffic_k_march2_scaled_f64_unit_tet_l8.txt")
CSRC = os.path.join(ROOT, "paper_1709_06793_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources the interior kernel and its launch grid come from
KERNEL_SOURCES = ("hhg_kernels.hip", "hhg_march.h", "hhg_lattice.h", "hhg_internal.h", "hhg_ctx.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(PROFILE):
        return None
    kv = {}
    for line in open(PROFILE):
        if ":" in line and not line.startswith("#"):
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_op(fn, steps, warmup, torch):
    """Average ms per call over `steps` calls on the current stream (HIP events)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def lognormal_on_device(xyz, prm, torch):
    from hhg_inputs import lognormal_k_torch
    return lognormal_k_torch(xyz, prm, torch)


def host_description():
    """nproc, the CPU model (lscpu) and the threads the oracle may use: the
    box's CPU share (at most 16 threads for one GPU) whatever os.cpu_count()
    shows."""
    import subprocess
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except Exception:
        nproc = os.cpu_count()
    model = "unknown"
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    threads = max(1, min(len(os.sched_getaffinity(0)), 16, nproc))
    return {"nproc": nproc, "os_cpu_count": os.cpu_count(), "cpu_model": model, "threads": threads}


def cpu_baseline(host):
    """The oracle as it stands on this host's cores.

    * Matvec: the oracle's CSR assembly of the scaled operator on the unit
      tet at level 8 (the GPU workload: 2,731,135 unknowns, 15 entries per
      row), then the oracle's plain C CSR product (OpenMP, static schedule
      over rows) on all threads of the machine's CPU share: 20 untimed products,
      200 timed, median; and on one thread (20 timed).
    * Time to solution: the oracle's multigrid (scipy CSR products, one
      thread; V(2,2), Chebyshev, P1 transfer, dense coarse solve) on the
      6-tet cube at level 6 (250,047 unknowns), smooth k, b = M I_h f, from
      u = 0 to a 1e-8 relative residual; its solution continued to 1e-12
      is the reference the GPU's level-6 solves are compared with."""
    from hhg_inputs import unit_tet, kuhn_cube, lognormal_params, lognormal_k, smooth_k, manufactured_f
    from oracle import oracle as O
    X, T = unit_tet()
    t0 = time.perf_counter()
    m = O.Mesh(X, T, 8)
    k = lognormal_k(m.xyz, lognormal_params(1, 1.0, 0.1))
    op = O.make_operator(m, k, "scaled")
    t_asm = time.perf_counter() - t0
    nu = op.A.shape[0]
    th = host["threads"]
    times = O.spmv_bench(op, th, warm=20, reps=200)
    t1 = O.spmv_bench(op, 1, warm=2, reps=20)
    gd = nu / float(np.median(times)) / 1e9
    gd1 = nu / float(np.median(t1)) / 1e9
    nnz = op.A.nnz
    del op, m, k
    log(f"bench: oracle CSR SpMV {gd:.3f} GDoF/s on {th} threads, {gd1:.3f} on 1")
    # multigrid time to solution, C3 level 6
    X6, T6 = kuhn_cube()
    t0 = time.perf_counter()
    mg = O.Multigrid(X6, T6, 6, 2, kfun=smooth_k, modification=True)
    mesh = mg.meshes[6]
    b = O.assemble_mass(mesh) @ manufactured_f(mesh.xyz)
    b[mesh.dirichlet] = 0.0
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    u, hist = mg.solve(b, tol=1e-8, maxit=100)
    t_solve = time.perf_counter() - t0
    uref = u.copy()
    op6 = mg.ops[6]
    nb = np.linalg.norm(b[mesh.unknowns])
    for _ in range(40):
        if np.linalg.norm(op6.residual(b, uref)[mesh.unknowns]) <= 1e-12 * nb:
            break
        uref = mg.vcycle(6, b, uref)
    out = {"value": round(gd, 4), "unit": "GDoF/s", "cores": th, "kind": "oracle",
           "sample": f"unit tet level 8 ({nu} unknowns, {nnz} stored entries; the GPU workload itself): the "
                     f"oracle's CSR matrix of the scaled operator (assembled in {t_asm:.1f} s by its element "
                     f"loops), plain C CSR product with OpenMP on {th} threads, median of 200 after 20 "
                     f"untimed; {nu * 200 / gd / 1e9:.1f} s of products",
           "single_thread_gdofs": round(gd1, 4),
           "host": host,
           "multigrid_c3_level6": {
               "unknowns": int(len(mesh.unknowns)), "seconds_to_1e-8": round(t_solve, 3),
               "setup_seconds": round(t_setup, 2), "iterations": len(hist) - 1,
               "rel_residual": float(f"{hist[-1]:.3g}"),
               "threads": 1,
               "note": "oracle multigrid, scipy CSR products (one thread), V(2,2) Chebyshev, from u = 0"}}
    return out, (mesh.xyz, uref)


def c3_solves(hhg, torch, oracle_ref=None):
    """The 6-tet Kuhn cube at levels 5-8 with smooth k and the manufactured
    solution u* = sin(pi x) sin(pi y) sin(pi z), b = M I_h f (consistent mass
    on the Freudenthal grid): FP64 and FP32-in-FP64 multigrid, V(2,2)
    Chebyshev, from u = 0 to a 1e-8 relative residual.  Each record states
    the discretisation error (discrete nodal L2 error against u*) and, at
    level 6, the error against the oracle's solution of the same system."""
    from hhg_inputs import kuhn_cube, smooth_k, manufactured_u, manufactured_f, kuhn_cube_mass_rhs
    X, T = kuhn_cube()
    out = {"cycle": "V(2,2)", "tol": 1e-8}
    prev = None
    for level in (5, 6, 7, 8):
        log(f"bench: C3 level {level}")
        ctx = hhg.Context(X, T, level)
        xyz, dirichlet = ctx.node_coords(level)
        ctx.set_coefficient(smooth_k(xyz))
        b = kuhn_cube_mass_rhs(xyz, level, manufactured_f)
        b[dirichlet] = 0.0
        fd = ctx.from_canonical(level, torch.tensor(b, device="cuda"))
        ustar = manufactured_u(xyz)
        h = 0.5 ** level
        rec = {"unknowns": ctx.sizes(level)["n_unknowns"]}
        for name, mode in (("f64", hhg.SOLVE_F64), ("mixed", hhg.SOLVE_MIXED)):
            best = None
            for _ in range(2):
                u = ctx.vector(level)
                torch.cuda.synchronize()
                st = ctx.solve(level, fd, u, mode=mode, tol=1e-8, max_iter=100)
                if best is None or st["seconds"] < best["seconds"]:
                    best, ub = st, u
            uh = ctx.to_canonical(level, ub).cpu().numpy()
            e = uh - ustar
            r = {k2: (float(f"{v:.4g}") if isinstance(v, float) else v) for k2, v in best.items()}
            r["nodal_l2_error"] = float(f"{np.sqrt(h ** 3 * np.sum(e[~dirichlet] ** 2)):.5g}")
            if oracle_ref is not None and level == 6:
                oxyz, ouref = oracle_ref
                # match nodes by coordinates (both sides number nodes their own way)
                key = lambda x: np.rint(x * 2 ** level).astype(np.int64) @ np.array([1, 1 << 10, 1 << 20])
                order_o = np.argsort(key(oxyz))
                order_g = np.argsort(key(xyz))
                a, c = uh[order_g], ouref[order_o]
                r["error_vs_oracle_solution"] = float(f"{np.linalg.norm(a - c) / np.linalg.norm(c):.3g}")
            rec[name] = r
            log(f"bench: C3 level {level} {name}: {r}")
        if prev is not None:
            rec["nodal_l2_eoc"] = round(float(np.log2(prev / rec["f64"]["nodal_l2_error"])), 3)
        prev = rec["f64"]["nodal_l2_error"]
        out[f"level{level}"] = rec
        ctx.close()
        del ctx, fd, u, ub
        torch.cuda.empty_cache()
    return out


def kuhn48_applies(hhg, torch, steps, solves=True, applies=True):
    """HBM-resident working set: 48 Kuhn tets, level 8 (133M unknowns): apply
    throughputs and/or multigrid time to solution.  The solves use coarse
    coefficients averaged geometrically from the finest level
    (HHG_FLAG_COARSE_K_GEOMETRIC: the field is rough) and the default coarse
    level (3: 3375 unknowns); solves with k sampled at the coarse nodes are
    reported beside them."""
    from hhg_inputs import kuhn_cube_2x2x2, lognormal_params
    level = 8
    log("bench: 48-tet cube level 8")
    X, T = kuhn_cube_2x2x2()
    ctx = hhg.Context(X, T, level, hhg.FLAG_COARSE_K_GEOMETRIC)
    xyz, dirichlet = ctx.node_coords(level)
    prm2 = lognormal_params(2, 1.5, 0.05)
    k = lognormal_on_device(xyz, prm2, torch)
    ctx.set_coefficient(k)
    del k
    sz = ctx.sizes(level)
    nu48 = sz["n_unknowns"]
    f = torch.tensor(prm2["rng"].uniform(-1, 1, xyz.shape[0]), device="cuda")
    f[torch.tensor(dirichlet, device="cuda")] = 0.0
    if applies:
        from hhg_inputs import tensor_fields_torch
        ctx.set_tensor_coefficient(tensor_fields_torch(xyz, torch))
        torch.cuda.empty_cache()
    del xyz
    f64 = ctx.from_canonical(level, f)
    del f
    y = ctx.vector(level)
    out = {"unknowns": nu48,
           "note": "48 Kuhn macro tets (2x2x2 cubes), lognormal sigma 1.5, l_c 0.05, seed 2; "
                   "3.3 GB FP64 working set, HBM-resident"}
    f32 = None
    if applies:
        steps48 = max(10, steps // 10)
        m1 = time_op(lambda: ctx.apply_scaled(level, f64, y), steps48, 3, torch)
        f32 = f64.float()
        y32 = ctx.vector(level, torch.float32)
        m2 = time_op(lambda: ctx.apply_scaled(level, f32, y32), steps48, 3, torch)
        m3 = time_op(lambda: ctx.apply_nodal(level, f64, y), steps48, 3, torch)
        m4 = time_op(lambda: ctx.apply_nodal(level, f32, y32), steps48, 3, torch)
        # primitive-mixed operator, nodal rows on macro vertices and edges
        m5 = time_op(lambda: ctx.apply_mixed(level, f64, y, hhg.PRIM_VERTICES | hhg.PRIM_EDGES), steps48, 3, torch)
        m6 = time_op(lambda: ctx.apply_mixed(level, f32, y32, hhg.PRIM_VERTICES | hhg.PRIM_EDGES), steps48, 3, torch)
        # tensor coefficient: every component scaled (interior rows from the
        # seven direction-pair fields), and every component nodally integrated
        # (the six component fields)
        m9 = time_op(lambda: ctx.apply_tensor(level, f64, y), steps48, 3, torch)
        m10 = time_op(lambda: ctx.apply_tensor(level, f32, y32), steps48, 3, torch)
        m11 = time_op(lambda: ctx.apply_tensor_nodal(level, f64, y), steps48, 3, torch)
        m12 = time_op(lambda: ctx.apply_tensor_nodal(level, f32, y32), steps48, 3, torch)
        # stored stencils (15 coefficients per row): the memory-bound baseline
        ctx.store_stencils(level)
        m7 = time_op(lambda: ctx.apply_stored(level, f64, y), steps48, 3, torch)
        m8 = time_op(lambda: ctx.apply_stored(level, f32, y32), steps48, 3, torch)
        del y32
        out.update({
            "tensor_f64_gdofs": round(nu48 / m9 / 1e6, 2),
            "tensor_f64_hbm_frac": round(72 * nu48 / m9 / 1e6 / HBM_PEAK_GBS, 4),
            "tensor_f32_gdofs": round(nu48 / m10 / 1e6, 2),
            "tensor_f32_hbm_frac": round(36 * nu48 / m10 / 1e6 / HBM_PEAK_GBS, 4),
            "tensor_nodal_f64_gdofs": round(nu48 / m11 / 1e6, 2),
            "tensor_nodal_f64_hbm_frac": round(64 * nu48 / m11 / 1e6 / HBM_PEAK_GBS, 4),
            "tensor_nodal_f32_gdofs": round(nu48 / m12 / 1e6, 2),
            "tensor_nodal_f32_hbm_frac": round(32 * nu48 / m12 / 1e6 / HBM_PEAK_GBS, 4),
            "stored_f64_gdofs": round(nu48 / m7 / 1e6, 2),
            "stored_f64_hbm_frac": round(136 * nu48 / m7 / 1e6 / HBM_PEAK_GBS, 4),
            "stored_f32_gdofs": round(nu48 / m8 / 1e6, 2),
            "stored_f32_hbm_frac": round(68 * nu48 / m8 / 1e6 / HBM_PEAK_GBS, 4),
            "scaled_f64_gdofs": round(nu48 / m1 / 1e6, 2),
            "scaled_f64_hbm_frac": round(BYTES_PER_DOF["f64"] * nu48 / m1 / 1e6 / HBM_PEAK_GBS, 4),
            "scaled_f32_gdofs": round(nu48 / m2 / 1e6, 2),
            "scaled_f32_hbm_frac": round(BYTES_PER_DOF["f32"] * nu48 / m2 / 1e6 / HBM_PEAK_GBS, 4),
            "nodal_f64_gdofs": round(nu48 / m3 / 1e6, 2),
            "nodal_f32_gdofs": round(nu48 / m4 / 1e6, 2),
            "mixed_vertices_edges_f64_gdofs": round(nu48 / m5 / 1e6, 2),
            "mixed_vertices_edges_f32_gdofs": round(nu48 / m6 / 1e6, 2)})
    if solves:
        def run_solves(c, cases):
            res = {}
            for name, mode, tol in cases:
                best = None
                for _ in range(2):
                    uu = c.vector(level)
                    torch.cuda.synchronize()
                    st = c.solve(level, f64, uu, mode=mode, tol=tol, max_iter=200)
                    if best is None or st["seconds"] < best["seconds"]:
                        best = st
                    del uu
                res[name] = {k2: (float(f"{v:.4g}") if isinstance(v, float) else v) for k2, v in best.items()}
                log(f"bench: solve {name}: {best}")
            return res
        res = run_solves(ctx, (("f64", hhg.SOLVE_F64, 1e-8), ("mixed", hhg.SOLVE_MIXED, 1e-8),
                               ("f64_1e-10", hhg.SOLVE_F64, 1e-10), ("mixed_1e-10", hhg.SOLVE_MIXED, 1e-10)))
        res["coarse_level"] = ctx.level_info(level)["coarse_level"]
        res["coarse_k"] = "geometric full-weighting averages"
        out["vcycle_solves"] = res
        del ctx
        torch.cuda.empty_cache()
        # the same solves with k sampled at the coarse nodes
        ctx = hhg.Context(X, T, level)
        xyz2, _ = ctx.node_coords(level)
        k = lognormal_on_device(xyz2, lognormal_params(2, 1.5, 0.05), torch)
        del xyz2
        ctx.set_coefficient(k)
        del k
        res2 = run_solves(ctx, (("f64_1e-10", hhg.SOLVE_F64, 1e-10), ("mixed_1e-10", hhg.SOLVE_MIXED, 1e-10)))
        res2["coarse_level"] = ctx.level_info(level)["coarse_level"]
        res2["coarse_k"] = "sampled at the coarse nodes"
        out["vcycle_solves_sampled_coarse_k"] = res2
    del ctx, f64, y, f32
    torch.cuda.empty_cache()
    return out

def learned_solves(hhg, torch):
    """Time to a 1e-8 relative residual on a held-out learned-smoother field
    (6-tet Kuhn cube, level 8, 16.6M unknowns, field seed 1000): the learned
    smoother (FP32 cycles, trained weights shipped with the package), plain
    Chebyshev FP32-in-FP64 and plain FP64 multigrid; best of two runs each."""
    from hhg_inputs import kuhn_cube, lognormal_params, lognormal_k
    from paper_1709_06793_amd import learned_train as LT
    level = 8
    log("bench: learned smoother, 6-tet cube level 8, field 1000")
    X, T = kuhn_cube()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    prm = lognormal_params(1000)
    ctx.set_coefficient(lognormal_k(xyz, prm))
    f = prm["rng"].uniform(-1, 1, xyz.shape[0])
    f[dirichlet] = 0.0
    fd = ctx.from_canonical(level, torch.tensor(f, device="cuda"))
    w, meta = LT.load_weights()
    ctx.learned_set_weights(w)
    ctx.learned_set_fallback(1.0, 1.05)
    out = {"unknowns": ctx.sizes(level)["n_unknowns"], "field_seed": 1000,
           "sigma": round(prm["sigma"], 4), "corr_len": round(prm["corr_len"], 4), "tol": 1e-8}
    for name, mode in (("learned", hhg.SOLVE_LEARNED), ("chebyshev_mixed", hhg.SOLVE_MIXED),
                       ("chebyshev_f64", hhg.SOLVE_F64)):
        best = None
        for _ in range(2):
            u = ctx.vector(level)
            torch.cuda.synchronize()
            st = ctx.solve(level, fd, u, mode=mode, tol=1e-8, max_iter=200)
            if best is None or st["seconds"] < best["seconds"]:
                best = st
        out[name] = {k2: (float(f"{v:.4g}") if isinstance(v, float) else v) for k2, v in best.items()}
        log(f"bench: {name}: {best}")
    del ctx
    torch.cuda.empty_cache()
    return out


def learned_held_out(hhg, torch, seeds=range(1000, 1032)):
    """The 32 held-out learned-smoother fields (seeds 1000-1031: sigma ~
    U(0.5, 2), correlation length ~ U(0.05, 0.3)) on the 6-tet cube at level
    8, re-timed in this run: time to a 1e-8 relative residual with the
    learned smoother (shipped weights, default fallback), plain Chebyshev
    FP32-in-FP64 and plain FP64; one solve each per field."""
    from hhg_inputs import kuhn_cube, lognormal_params
    from paper_1709_06793_amd import learned_train as LT
    level = 8
    log("bench: learned smoother on 32 held-out fields, 6-tet cube level 8")
    X, T = kuhn_cube()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    w, _ = LT.load_weights()
    cols = {name: {"iterations": [], "seconds": [], "fallback": [], "rho": []}
            for name in ("learned", "chebyshev_mixed", "chebyshev_f64")}
    dmask = torch.tensor(dirichlet, device="cuda")
    for seed in seeds:
        prm = lognormal_params(seed)
        ctx.set_coefficient(lognormal_on_device(xyz, prm, torch))
        f = torch.tensor(prm["rng"].uniform(-1, 1, xyz.shape[0]), device="cuda")
        f[dmask] = 0.0
        fd = ctx.from_canonical(level, f)
        ctx.learned_set_weights(w)
        ctx.learned_set_fallback(1.0, 1.05)
        for name, mode in (("learned", hhg.SOLVE_LEARNED), ("chebyshev_mixed", hhg.SOLVE_MIXED),
                           ("chebyshev_f64", hhg.SOLVE_F64)):
            u = ctx.vector(level)
            torch.cuda.synchronize()
            st = ctx.solve(level, fd, u, mode=mode, tol=1e-8, max_iter=200)
            if st["rel_residual"] > 1e-8:
                raise RuntimeError(f"field {seed} {name}: no convergence {st}")
            for key in cols[name]:
                cols[name][key].append(st[key])
    out = {"fields": len(list(seeds)), "unknowns": ctx.sizes(level)["n_unknowns"], "tol": 1e-8}
    for name, c in cols.items():
        out[name] = {"mean_iterations": round(float(np.mean(c["iterations"])), 3),
                     "mean_seconds": round(float(np.mean(c["seconds"])), 5),
                     "median_rho": round(float(np.median(c["rho"])), 4),
                     "fallbacks": int(np.sum(c["fallback"]))}
    li, ci = np.array(cols["learned"]["iterations"]), np.array(cols["chebyshev_mixed"]["iterations"])
    ls, cs = np.array(cols["learned"]["seconds"]), np.array(cols["chebyshev_mixed"]["seconds"])
    out["learned_fewer_cycles_than_chebyshev"] = int((li < ci).sum())
    out["learned_faster_than_chebyshev_mixed"] = int((ls < cs).sum())
    out["learned_faster_than_f64"] = int((ls < np.array(cols["chebyshev_f64"]["seconds"])).sum())
    log(f"bench: held-out fields: {out}")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def scalar_form_solves(hhg, torch):
    """Ten V(3,3) cycles per operator as in the paper's 3D scalar comparison
    (Sec. 7.2: 6-tet unit cube, level 8 here = 16.6M unknowns,
    k = cos(m pi xyz) + 2 for m = 3 and 8; homogeneous Dirichlet data,
    f ~ U[-1,1]): stencil scaling everywhere, the primitive-mixed operator
    with nodal rows on macro vertices and edges ("scale Vol+Face") and nodal
    integration, FP64; best of two runs each (the first also builds the
    operator's diagonals and coarse inverse)."""
    from hhg_inputs import kuhn_cube, cosine_k
    level = 8
    log("bench: scalar operator comparison, 6-tet cube level 8")
    X, T = kuhn_cube()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    f = np.random.default_rng(6).uniform(-1, 1, xyz.shape[0])
    f[dirichlet] = 0.0
    fd = ctx.from_canonical(level, torch.tensor(f, device="cuda"))
    out = {"unknowns": ctx.sizes(level)["n_unknowns"], "cycles": 10, "cycle": "V(3,3)"}
    for m in (3, 8):
        ctx.set_coefficient(cosine_k(xyz, m))
        res = {}
        for name, form in (("scaled", "scaled"), ("scale_vol_face", "mixed"), ("nodal", "nodal")):
            best = None
            for _ in range(2):
                u = ctx.vector(level)
                torch.cuda.synchronize()
                st = ctx.solve_form(level, fd, u, form=form, nodal_primitives=hhg.PRIM_VERTICES | hhg.PRIM_EDGES,
                                    tol=0.0, max_iter=10, pre=3, post=3)
                if best is None or st["seconds"] < best["seconds"]:
                    best = st
                del u
            res[name] = {k2: (float(f"{v:.4g}") if isinstance(v, float) else v) for k2, v in best.items()}
            log(f"bench: m={m} {name}: {best}")
        res["relative_tts_scaled"] = round(res["scaled"]["seconds"] / res["nodal"]["seconds"], 3)
        res["relative_tts_scale_vol_face"] = round(res["scale_vol_face"]["seconds"] / res["nodal"]["seconds"], 3)
        out[f"m{m}"] = res
    del ctx, fd
    torch.cuda.empty_cache()
    return out


def applies_2d(torch, steps):
    """The 2D variant (Sec. 4.1's exact MA2): the non-Delaunay macro square
    (8 triangles, four with an obtuse angle) at level 11 (16.8M nodes),
    sigmoid k with eta = 1000 and slope m = 2000 (steep enough that MA2 still
    replaces factors at this level); FP64 / FP32 scaled and FP64 nodal
    applies."""
    from hhg_inputs import square_nondelaunay8, sigmoid_k
    from paper_1709_06793_amd import hhg2d
    level = 11
    log("bench: 2D applies, non-Delaunay square level 11")
    X, T = square_nondelaunay8()
    t0 = time.time()
    ctx = hhg2d.Context2D(X, T, level)
    xy, dirichlet = ctx.node_coords()
    ctx.set_coefficient(sigmoid_k(xy, 1000.0, m=2000.0))
    setup_s = time.time() - t0
    sz = ctx.sizes()
    u = np.random.default_rng(3).uniform(-1, 1, len(xy))
    u[dirichlet] = 0.0
    u64 = ctx.from_canonical(torch.tensor(u, device="cuda"))
    u32 = u64.float()
    y64, y32 = ctx.vector(), ctx.vector(torch.float32)
    m1 = time_op(lambda: ctx.apply_scaled(u64, y64), steps, 5, torch)
    m2 = time_op(lambda: ctx.apply_scaled(u32, y32), steps, 5, torch)
    m3 = time_op(lambda: ctx.apply_nodal(u64, y64), steps, 5, torch)
    nu = sz["n_unknowns"]
    out = {"nodes": sz["n_nodes"], "unknowns": nu, "modified_edges": sz["n_modified"],
           "setup_s": round(setup_s, 2),
           "scaled_f64_gdofs": round(nu / m1 / 1e6, 2),
           "scaled_f64_hbm_frac": round(24 * nu / m1 / 1e6 / HBM_PEAK_GBS, 4),
           "scaled_f32_gdofs": round(nu / m2 / 1e6, 2),
           "nodal_f64_gdofs": round(nu / m3 / 1e6, 2)}
    ctx.close()
    torch.cuda.empty_cache()
    return out


def tensor_solves(hhg, torch):
    """Time to a 1e-9 relative residual with the tensor operator (the
    tensor-coefficient comparison of Sec. 7.3: 12 macro tets around the cube
    centre, level 8, 33.4M unknowns, that comparison's polynomial SPD K,
    homogeneous Dirichlet data, f ~ U[-1,1]): V(3,3) cycles with every
    component scaled and with every component nodally integrated, FP64 and
    FP32-in-FP64; best of two runs each (the first run also builds the form's
    diagonals and coarse inverse)."""
    from hhg_inputs import cube12, polynomial_tensor_fields_torch
    level = 8
    log("bench: tensor solves, 12-tet cube level 8")
    X, T = cube12()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    ctx.set_tensor_coefficient(polynomial_tensor_fields_torch(xyz, torch))
    f = np.random.default_rng(5).uniform(-1, 1, xyz.shape[0])
    f[dirichlet] = 0.0
    fd = ctx.from_canonical(level, torch.tensor(f, device="cuda"))
    del xyz
    out = {"unknowns": ctx.sizes(level)["n_unknowns"], "tol": 1e-9, "cycle": "V(3,3)",
           "K": "polynomial SPD tensor of the paper's tensor comparison"}
    for form in ("scaled", "nodal"):
        for mname, mode in (("f64", hhg.SOLVE_F64), ("mixed", hhg.SOLVE_MIXED)):
            best = None
            for _ in range(2):
                u = ctx.vector(level)
                torch.cuda.synchronize()
                st = ctx.solve_tensor(level, fd, u, form=form, mode=mode, tol=1e-9, max_iter=200, pre=3, post=3)
                if best is None or st["seconds"] < best["seconds"]:
                    best = st
                del u
            out[f"{form}_{mname}"] = {k2: (float(f"{v:.4g}") if isinstance(v, float) else v)
                                      for k2, v in best.items()}
            log(f"bench: tensor {form} {mname}: {best}")
    for mname in ("f64", "mixed"):
        out[f"relative_tts_{mname}"] = round(out[f"scaled_{mname}"]["seconds"] / out[f"nodal_{mname}"]["seconds"], 3)
    del ctx, fd
    torch.cuda.empty_cache()
    return out


def blending_solves(hhg, torch, levels=(3, 4, 5, 6, 7)):
    """The blending example of Sec. 7.4 on one GPU: the half cylinder mantle's
    reference box in 80 Kuhn blocks (480 tets), coefficient (1 + z) K with K
    from the mapping, the manufactured solution made zero on the boundary,
    b = M I_h f; V(3,3) to a 1e-8 relative residual (as in that example) with
    every tensor component scaled and with every component nodally
    integrated, FP64 (best of two runs).  Per level: unknowns, nodal L2 error
    against u*, its order, the multigrid rate and the times."""
    from hhg_inputs import (CYLINDER_BOX, cylinder_reference_box, kuhn_box_mass_rhs, cylinder_tensor_fields_torch,
                            cylinder_u, cylinder_f)
    blocks = (1, 8, 10)
    X, T = cylinder_reference_box(blocks)
    lo, hi = CYLINDER_BOX
    out = {"macro_tets": int(T.shape[0]), "cycle": "V(3,3)", "tol": 1e-8, "precision": "f64"}
    prev = {}
    for level in levels:
        log(f"bench: blending level {level}")
        ctx = hhg.Context(X, T, level)
        xyz, dirichlet = ctx.node_coords(level)
        ctx.set_tensor_coefficient(cylinder_tensor_fields_torch(xyz, torch))
        b = kuhn_box_mass_rhs(xyz, level, cylinder_f, blocks, lo, hi)
        b[dirichlet] = 0.0
        fd = ctx.from_canonical(level, torch.tensor(b, device="cuda"))
        del b
        ustar = cylinder_u(xyz)
        vol = float(np.prod((np.asarray(hi) - np.asarray(lo)) / (np.asarray(blocks) * 2 ** level)))
        rec = {"unknowns": ctx.sizes(level)["n_unknowns"]}
        for form in ("nodal", "scaled"):
            best, ub = None, None
            for _ in range(2):
                u = ctx.vector(level)
                torch.cuda.synchronize()
                st = ctx.solve_tensor(level, fd, u, form=form, mode=hhg.SOLVE_F64, tol=1e-8, max_iter=100,
                                      pre=3, post=3)
                if best is None or st["seconds"] < best["seconds"]:
                    best, ub = st, u
            e = ctx.to_canonical(level, ub).cpu().numpy() - ustar
            r = {"error": float(f"{np.sqrt(vol * np.sum(e[~dirichlet] ** 2)):.4g}"),
                 "rho": round(best["rho"], 3), "iterations": best["iterations"],
                 "seconds": float(f"{best['seconds']:.4g}"), "status": best["status"]}
            if form in prev:
                r["eoc"] = round(float(np.log2(prev[form] / r["error"])), 3)
            prev[form] = r["error"]
            rec[form] = r
            log(f"bench: blending level {level} {form}: {r}")
            del ub, u
        rec["relative_tts"] = round(rec["scaled"]["seconds"] / rec["nodal"]["seconds"], 3)
        out[f"level{level}"] = rec
        ctx.close()
        del ctx, fd, xyz, ustar
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="value only: skip the context measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--k48-apply-only", action="store_true",
                    help="only time the 48-tet level-8 applies (tuning runs)")
    ap.add_argument("--applies-2d", action="store_true", help="only the 2D applies (non-Delaunay square, level 11)")
    ap.add_argument("--form-solves", action="store_true",
                    help="only the scalar operator comparison (6-tet cube, level 8, ten V(3,3) cycles)")
    ap.add_argument("--tensor-solves", action="store_true",
                    help="only the tensor-operator solves (12-tet cube, level 8)")
    ap.add_argument("--c3-solves", action="store_true", help="only the 6-tet cube solves at levels 5-8")
    ap.add_argument("--held-out", action="store_true", help="only the 32 held-out learned-smoother fields")
    ap.add_argument("--blending", action="store_true", help="only the blending example's solves (Sec. 7.4)")
    ap.add_argument("--k48-solves", action="store_true",
                    help="only run the 48-tet level-8 V-cycle solves (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "multi-GPU execution is not implemented: the benchmark runs on one GPU (--gpus 1)"}))
        sys.exit(2)
    import torch
    from hhg_inputs import unit_tet, kuhn_cube, kuhn_cube_2x2x2, lognormal_params, smooth_k
    from paper_1709_06793_amd import hhg

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8}))
        return

    if args.k48_apply_only:
        print(json.dumps(kuhn48_applies(hhg, torch, args.steps, solves=False)))
        return
    if args.applies_2d:
        print(json.dumps(applies_2d(torch, args.steps)))
        return
    if args.form_solves:
        print(json.dumps(scalar_form_solves(hhg, torch)))
        return
    if args.tensor_solves:
        print(json.dumps(tensor_solves(hhg, torch)))
        return
    if args.k48_solves:
        print(json.dumps(kuhn48_applies(hhg, torch, args.steps, solves=True, applies=False)))
        return
    if args.c3_solves:
        print(json.dumps(c3_solves(hhg, torch)))
        return
    if args.held_out:
        print(json.dumps(learned_held_out(hhg, torch)))
        return
    if args.blending:
        print(json.dumps(blending_solves(hhg, torch)))
        return

    # ---------------- main workload: unit tet, level 8, lognormal k
    level = 8
    X, T = unit_tet()
    log("bench: building unit tet level 8 context")
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    prm = lognormal_params(1, 1.0, 0.1)
    k = lognormal_on_device(xyz, prm, torch)
    u = torch.tensor(prm["rng"].uniform(-1, 1, xyz.shape[0]), device="cuda")
    u[torch.tensor(dirichlet, device="cuda")] = 0.0
    ctx.set_coefficient(k)
    sz = ctx.sizes(level)
    nu = sz["n_unknowns"]
    u64 = ctx.from_canonical(level, u)
    y64 = ctx.vector(level)
    log(f"bench: unknowns {nu}, timing {args.steps} applies")
    ms = time_op(lambda: ctx.apply_scaled(level, u64, y64), args.steps, args.warmup, torch)
    value = nu / (ms * 1e-3) / 1e9
    # the interior kernel, timed by a pair of HIP events that its launch
    # stamps on the stream it runs on (hipExtLaunchKernel: dispatch to
    # completion, no separate event commands; the unit tet has no inter-tet
    # rows and no modified edges, so each apply is this one kernel): (a) back to back, as
    # the timed steps run, with the 69 MB working set resident in the 256 MB
    # last-level cache; (b) with a 1 GiB read between launches, so that the
    # kernel reads u and k from HBM: the roofline figure.  The flush is a read
    # (a sum over the buffer), so the caches hold clean lines and the kernel
    # pays for no write-back of the flush's own data.
    ctx.set_timing(True)
    time_op(lambda: ctx.apply_scaled(level, u64, y64), args.steps, 0, torch)
    k_ms_tot, k_n = ctx.read_timing()
    k_ms_warm = k_ms_tot / k_n
    flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for q in range(args.steps):
        flush.sum()
        ctx.apply_scaled(level, u64, y64)
    torch.cuda.synchronize()
    k_ms_tot, k_n = ctx.read_timing()
    ctx.set_timing(False)
    k_ms = k_ms_tot / k_n
    # measured copy roof: a 1 GiB device-to-device copy (reads and writes)
    dst = torch.empty_like(flush)
    copy_ms = time_op(lambda: dst.copy_(flush), 10, 2, torch)
    copy_gbs = 2 * flush.numel() * 8 / (copy_ms * 1e-3) / 1e9
    # and a copy moving the kernel's algorithmic bytes (half read, half
    # written), timed the same way as the kernel: after a 1 GiB read
    ncp = BYTES_PER_DOF["f64"] * nu // 16
    src_s, dst_s = torch.ones(ncp, dtype=torch.float64, device="cuda"), torch.empty(ncp, dtype=torch.float64,
                                                                                   device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for q in range(args.steps):
        flush.sum()
        ev[q][0].record()
        dst_s.copy_(src_s)
        ev[q][1].record()
    torch.cuda.synchronize()
    copy_small_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    copy_small_gbs = 16 * ncp / (copy_small_ms * 1e-3) / 1e9
    del flush, dst, src_s, dst_s
    torch.cuda.empty_cache()
    achieved = BYTES_PER_DOF["f64"] * nu / (k_ms * 1e-3) / 1e9
    n_mod = ctx.level_info(level)["n_modified"]
    traffic = measured_traffic()
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "unit macro tet (0,0,0),(1,0,0),(0,1,0),(0,0,1), level 8 "
                               f"({sz['n_slots']} slots, {nu} unknowns), lognormal k (32 Fourier modes, "
                               "sigma 1, correlation length 0.1, seed 1), u ~ U[-1,1]: one FP64 "
                               "scaled-stencil apply per step, applies back to back (the 69 MB working set "
                               "stays in the 256 MB last-level cache between steps)",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_counter": "FETCH_SIZE + WRITE_SIZE per launch (L2 to fabric: what HBM serves "
                                        "when the last-level cache holds none of the inputs), scaled by the copy "
                                        "calibration; null when taken on other kernel sources",
                     "kernel": "k_march2<double, MODE_APPLY, scaled> (interior rows, two per lane; the unit "
                               "tet has no inter-tet rows)",
                     "timing": "mean duration per launch from the HIP event pair each launch stamps on its "
                               "stream (hipExtLaunchKernel), a 1 GiB read between launches (inputs read from "
                               "HBM); the copies are timed with events recorded around them",
                     "kernel_ms": round(k_ms, 5),
                     "kernel_ms_back_to_back": round(k_ms_warm, 5),
                     "frac_back_to_back": round(BYTES_PER_DOF["f64"] * nu / (k_ms_warm * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                                4),
                     "copy_roof_gbs": round(copy_gbs, 1),
                     "frac_of_copy_roof": round(achieved / copy_gbs, 4),
                     "copy_same_bytes_after_flush_gbs": round(copy_small_gbs, 1),
                     "frac_of_copy_same_bytes_after_flush": round(achieved / copy_small_gbs, 4),
                     "algorithmic_bytes_per_launch": BYTES_PER_DOF["f64"] * nu,
                     "other_kernels": ("none" if n_mod == 0 else
                                       f"k_correction<double> ({n_mod} modified edges) once per apply")},
    }
    extra = {}
    if not args.quick:
        # FP32 apply and the nodal-integration kernel on the same workload
        u32 = u64.float()
        y32 = ctx.vector(level, torch.float32)
        ms32 = time_op(lambda: ctx.apply_scaled(level, u32, y32), args.steps, args.warmup, torch)
        msn = time_op(lambda: ctx.apply_nodal(level, u64, y64), args.steps, args.warmup, torch)
        msn32 = time_op(lambda: ctx.apply_nodal(level, u32, y32), args.steps, args.warmup, torch)
        r64 = ctx.vector(level)
        msr = time_op(lambda: ctx.residual(level, y64, u64, r64), args.steps, args.warmup, torch)
        # FP32 interior kernel with a 1 GiB read between launches
        flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ctx.set_timing(True)
        for q in range(args.steps):
            flush.sum()
            ctx.apply_scaled(level, u32, y32)
        torch.cuda.synchronize()
        k32_tot, k32_n = ctx.read_timing()
        ctx.set_timing(False)
        del flush
        k32_ms = k32_tot / k32_n
        extra["unit_tet_l8"] = {
            "scaled_f64_gdofs": round(value, 2), "scaled_f32_gdofs": round(nu / ms32 / 1e6, 2),
            "nodal_f64_gdofs": round(nu / msn / 1e6, 2), "nodal_f32_gdofs": round(nu / msn32 / 1e6, 2),
            "scaled_over_nodal_f64": round(msn / ms, 3), "scaled_over_nodal_f32": round(msn32 / ms32, 3),
            "residual_f64_gdofs": round(nu / msr / 1e6, 2),
            "scaled_f32_frac_back_to_back": round(BYTES_PER_DOF["f32"] * nu / ms32 / 1e6 / HBM_PEAK_GBS, 4),
            "scaled_f32_kernel_ms_cold": round(k32_ms, 5),
            "scaled_f32_hbm_frac_cold": round(BYTES_PER_DOF["f32"] * nu / k32_ms / 1e6 / HBM_PEAK_GBS, 4),
            "note": "back-to-back rates: the working set (69 MB FP64) stays in the 256 MB last-level cache; "
                    "'cold': kernel duration with a 1 GiB read between launches (inputs from HBM)"}
        del ctx, u64, y64, u32, y32, r64
        torch.cuda.empty_cache()

        cpu_out, oracle_ref = (None, None)
        if not args.no_cpu:
            log("bench: CPU oracle baseline")
            cpu_out, oracle_ref = cpu_baseline(host_description())
        extra["c3_6tet"] = c3_solves(hhg, torch, oracle_ref)
        extra["kuhn48_l8"] = kuhn48_applies(hhg, torch, args.steps, solves=True)
        extra["learned_l8"] = learned_solves(hhg, torch)
        extra["learned_held_out_l8"] = learned_held_out(hhg, torch)
        extra["forms_6tet_l8"] = scalar_form_solves(hhg, torch)
        extra["square2d_l11"] = applies_2d(torch, args.steps)
        extra["tensor_cube12_l8"] = tensor_solves(hhg, torch)
        extra["blending_cylinder"] = blending_solves(hhg, torch)
    else:
        cpu_out = None
        if not args.no_cpu:
            log("bench: CPU oracle baseline")
            cpu_out, _ = cpu_baseline(host_description())
    out["extra"] = extra
    out["cpu_baseline"] = cpu_out
    print(json.dumps(out))


if __name__ == "__main__":
    main()
