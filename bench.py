#!/usr/bin/env python3
"""Benchmark of the energetic single-layer hot path on one MI355X.

One step = the whole path on the icosphere workload (radius 1, level 2,
320 triangles, T = 4, 32 slabs, interior time levels jittered by
+-0.2 dt, N = 30,720 panels), inputs resident in HBM:
  mesh ingest + panel geometry, causal cull + compaction, clip + inner
  quadrature + outer sum + causal-only store (every causal pair), FP64
  matvec, 16-RHS FP32 matrix-core product, potential at 1,000 shell points.
value = causal element-pairs assembled per second of step time.

Legs beside the step (same JSON line): mixed precision on the same mesh,
the 64-mesh batched workload (icospheres of levels 0-3 x 8-64 slabs,
seed 3) with 16-RHS products, serving on 8 resident meshes of that mix
(seed 5), the indirect solves (GMRES and marching-on-in-time), the
double-layer potential, and the oracle on the host cores.

Prints one JSON line.  --gpus > 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "causal element-pairs/s, FP64 vs mixed at rel.err≤1e-6; serving p50/p99 latency"
FP64_VECTOR_PEAK = 78.6e12      # MI355X dense FP64 vector FLOP/s
HBM_PEAK = 8.0e12               # MI355X HBM3E bytes/s
# Algorithmic work of the method (what the rule must compute, not the
# instructions a kernel issues), per unit:
#   one evaluation of L(phi): the four face quadratics (discriminant, one
#   square root and one quotient each), the interval logic and the r-measure
#   of the gaps, the node map and weight: 110 FLOP, plus one sin/cos pair;
#   one lit (outer point, panel) pair: apex data, face coefficients, the
#   phi-breakpoints (edge events, tangencies, asymptotes: about 14
#   arctangents / arccosines counted as one operation each): 414 FLOP.
C_NODE_FLOP = 110.0
C_SETUP_FLOP = 414.0
# A finer count of what the node kernels' formulas need, by the path that
# evaluates them (FMA = 2, add / mul = 1, divide / sqrt / sin / cos = 1):
# node map, weight and accumulation 12, sin + cos 2; one endpoint root 14;
# one face with both roots 16; r-measure of a gap 6.  One-gap recipe
# 12 + 2 + 2 x 14 + 6 = 48; two-gap recipe 12 + 2 + 4 x 14 + 2 x 6 = 82;
# full evaluation 12 + 2 + 4 x 16 + 5 x 6 = 108.  Reported beside the
# roofline, not in it.
FLOP_PER_L = {"recipe1": 48.0, "recipe2": 82.0, "full": 108.0}


def node_flops(counts):
    return sum(FLOP_PER_L[k] * counts.get(k, 0) for k in FLOP_PER_L)


# Bytes measured by rocprofv3 on this workload (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 per dispatch, factors from a plain 1 GiB copy in the same
# runs; L2 misses, an upper bound on HBM bytes), from
# profiles/node_stage_icosphere_L2_S32.md: per launch group of the FP64
# node stage, and summed over every kernel of one assembly.  Set to None
# whenever the kernels change until they are profiled again.
K_NODES_TRAFFIC_BYTES = 1.288e10
ASSEMBLY_TRAFFIC_BYTES = 3.083e11


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=1000)
    ap.add_argument("--cpu-rows", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-mesh batched leg")
    ap.add_argument("--no-solve", action="store_true", help="skip the indirect-solve legs")
    ap.add_argument("--no-dl", action="store_true", help="skip the double-layer leg")
    ap.add_argument("--no-litsearch", action="store_true", help="skip the lit-search timing leg")
    ap.add_argument("--direct", action="store_true", help="add the direct-method leg")
    ap.add_argument("--workload", choices=["icosphere", "batch"], default="icosphere",
                    help="icosphere: the 30,720-panel step (default); batch: only the 64-mesh "
                         "batched workload, as the main line")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-group", type=int, default=8, help="meshes per batch call")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=500, help="requests per arrival rate")
    ap.add_argument("--serve-unloaded", type=int, default=100, help="requests for the unloaded latency")
    ap.add_argument("--serve-rates", default="12,24,48", help="Poisson arrival rates, req/s")
    ap.add_argument("--serve-reps", type=int, default=2, help="independent runs per rate")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def cpu_baseline(mesh, nrows):
    """The oracle, untuned, on a bounded seeded sample of the rows."""
    import numpy as np
    import oracle
    rows = np.sort(np.random.default_rng(11).choice(mesh.nt, nrows, replace=False))
    oracle.assemble_rows(mesh.vtx, mesh.tets, rows=rows[:4])          # load + warm
    t0 = time.perf_counter()
    A = oracle.assemble_rows(mesh.vtx, mesh.tets, rows=rows)
    dt = time.perf_counter() - t0
    pairs = int(np.count_nonzero(A))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": pairs / dt, "unit": "causal element-pairs/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": model,
            "sample": "%d seeded rows x all %d columns (%d causal pairs) in %.2f s" %
                      (nrows, mesh.nt, pairs, dt)}


def serving_leg(args, ctx, stb):
    """Requests on 8 device-resident meshes through the continuous-batching
    server: the batched workload's mix generator (icospheres of levels 0-3 x
    8-64 slabs, T = 4, jitter +-0.2 dt) with seed 5, each mesh's causal-only
    store resident; half matvec (16 RHS ~ N(0,1)), half potential at P points,
    P log-uniform in [1e3, 1e5], |x| uniform in volume on [1.5, 3],
    t ~ U[0, T], density ~ N(0,1) (inputs drawn from per-mesh pools, so that
    hundreds of requests fit in host memory).  Unloaded latency from
    --serve-unloaded requests one at a time, then --serve-reps independent
    runs of --serve-requests Poisson arrivals at each rate; reported: every
    run's p50/p99 with its request count, and the highest rate whose p99 stays
    below twice the unloaded p99 in every run."""
    import threading
    import numpy as np
    from paper_2103_16841_amd import inputs
    meshes = inputs.batch_mix(count=8, seed=5)
    t0 = time.perf_counter()
    hs = [stb.Mesh(ctx, m.vtx, m.tets) for m in meshes]
    mats = [stb.assemble_V(ctx, h) for h in hs]
    t_asm = time.perf_counter() - t0
    print("serving: %d resident meshes, panels %s, causal pairs %s (%.1f s to assemble)" %
          (len(meshes), [m.nt for m in meshes], [A.n_causal for A in mats], t_asm),
          file=sys.stderr, flush=True)
    S = stb.Server(ctx, nslots=4)
    ids = [S.add_mesh(h, A) for h, A in zip(hs, mats)]
    rng = np.random.default_rng(5)
    pool_W = [[rng.standard_normal((m.nt, 16)) for _ in range(2)] for m in meshes]
    pool_w = [[rng.standard_normal(m.nt) for _ in range(2)] for m in meshes]
    pool_p = inputs.shell_points(200000, meshes[0].T, seed=55)

    def make(n):
        out = []
        for _ in range(n):
            i = int(rng.integers(len(meshes)))
            if rng.uniform() < 0.5:
                out.append(("matvec", i, pool_W[i][int(rng.integers(2))]))
            else:
                P = int(round(10 ** rng.uniform(3, 5)))
                o = int(rng.integers(0, pool_p.shape[0] - P + 1))
                out.append(("potential", i, (pool_w[i][int(rng.integers(2))], pool_p[o:o + P])))
        return out

    def submit(r):
        k, i, d = r
        return S.submit_matvec(ids[i], d) if k == "matvec" else S.submit_potential(ids[i], d[0], d[1])

    unl = []
    for r in make(args.serve_unloaded):
        unl.append(S.wait(submit(r))[1])
    unl_p50, unl_p99 = float(np.percentile(unl, 50)), float(np.percentile(unl, 99))
    print("serving unloaded (%d requests): p50 %.1f ms p99 %.1f ms" % (len(unl), 1e3 * unl_p50, 1e3 * unl_p99),
          file=sys.stderr, flush=True)
    sweep = []
    for rate in [float(x) for x in args.serve_rates.split(",")]:
        runs = []
        for rep in range(args.serve_reps):
            reqs = make(args.serve_requests)
            tickets, lat = [], []

            def waiter():
                k = 0
                while k < len(reqs):
                    while k >= len(tickets):
                        time.sleep(0.0005)
                    lat.append(S.wait(tickets[k])[1])
                    k += 1
            th = threading.Thread(target=waiter)
            th.start()
            gaps = rng.exponential(1.0 / rate, size=len(reqs))
            t0 = time.perf_counter()
            t_next = t0
            for r, g in zip(reqs, gaps):
                t_next += g
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets.append(submit(r))
            th.join()
            span = time.perf_counter() - t0
            runs.append({"requests": len(lat), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                         "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                         "throughput_req_s": len(reqs) / span})
            print("serving rate %g run %d: %d requests p50 %.1f ms p99 %.1f ms, %.1f req/s" %
                  (rate, rep, len(lat), runs[-1]["p50_ms"], runs[-1]["p99_ms"],
                   runs[-1]["throughput_req_s"]), file=sys.stderr, flush=True)
        sweep.append({"rate_req_s": rate, "runs": runs})
    S.close()
    for A in mats:
        A.close()
    ok = [x for x in sweep if all(r["p99_ms"] < 2e3 * unl_p99 for r in x["runs"])]
    best = max(ok, key=lambda x: x["rate_req_s"]) if ok else None
    return {"meshes": [m.nt for m in meshes], "causal_pairs": [int(A.n_causal) for A in mats],
            "mesh_mix": "batch mix generator, seed 5, levels 0-3 x 8-64 slabs",
            "assembly_s": t_asm, "slots": 4, "unloaded_requests": len(unl),
            "unloaded_p50_ms": 1e3 * unl_p50, "unloaded_p99_ms": 1e3 * unl_p99,
            "at_rate": best, "sweep": sweep,
            "requests": "50% matvec 16 RHS, 50% potential P log-uniform [1e3, 1e5]"}


def solve_leg(ctx, stb, mesh):
    """The indirect system (eq. df_ind) with the sphere's closed form:
    boundary data g(t) = 1/2 int_0^2 f(t - r) dr belongs to the time-only
    density f(t) = sin^2(pi t / 2) on [0, 2].  GMRES(100) to a relative
    residual of 1e-10 on the jittered bench mesh; on the same sphere
    unjittered (32 equal slabs), marching-on-in-time beside GMRES.  Errors of
    the solutions against f at the panel centroids."""
    import numpy as np
    import torch
    from paper_2103_16841_amd import inputs

    def F(s):
        c = np.clip(s, 0.0, 2.0)
        return 0.5 * c - np.sin(np.pi * c) / (2.0 * np.pi)

    def g(p):
        return 0.5 * (F(p[:, 0]) - F(p[:, 0] - 2.0))

    def exact(me):
        tc = me.vtx[me.tets][:, :, 0].mean(axis=1)
        return np.where((tc > 0) & (tc < 2), np.sin(0.5 * np.pi * tc) ** 2, 0.0)

    out = {}
    for key, me in (("jittered", mesh),
                    ("slabs", inputs.icosphere_mesh(level=2, S=32, T=4.0, jitter=0.0, seed=0))):
        m = stb.Mesh(ctx, me.vtx, me.tets)
        A = stb.assemble_V(ctx, m)
        b = stb.energetic_rhs(ctx, m, g)
        f = exact(me)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, its, rr = stb.solve_gmres(ctx, A, b, restart=100, maxit=20000, rtol=1e-10)
        dt = time.perf_counter() - t0
        r = {"gmres": {"products": its, "relres": rr, "ms": dt * 1e3,
                       "rel_l2_error_vs_exact_density": float(np.linalg.norm(x - f) / np.linalg.norm(f))}}
        if key == "slabs":
            t0 = time.perf_counter()
            xm, info = stb.solve_mot(ctx, m, A, b)
            dtm = time.perf_counter() - t0
            r["mot"] = {"ms": dtm * 1e3, **info,
                        "rel_l2_error_vs_exact_density": float(np.linalg.norm(xm - f) / np.linalg.norm(f)),
                        "rel_diff_vs_gmres": float(np.linalg.norm(xm - x) / np.linalg.norm(x))}
        r["mesh"] = me.name
        r["panels"] = me.nt
        out[key] = r
        A.close()
        m.close()
    return out


def lit_search_leg(ctx, stb, npts=32768, reps=3):
    """Exp. 1's timing question on this GPU: the lit search of npts points at
    t = T inside the unit ball (T = 5, icosphere levels 0-3 with 5-40 slabs)
    by the cluster tree and by the flat cull, as the potential's cull phase
    (HIP events, median of reps after one warm-up), per point, with the
    candidate pairs each produces and the lit pairs (equal for both)."""
    import numpy as np
    from paper_2103_16841_amd import inputs
    rows = []
    rng = np.random.default_rng(41)
    d = rng.standard_normal((npts, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = np.concatenate([np.full((npts, 1), 5.0), d * rng.uniform(0.0, 1.0, (npts, 1)) ** (1 / 3)], axis=1)
    for L in range(4):
        me = inputs.icosphere_mesh(level=L, S=5 * 2 ** L, T=5.0, jitter=0.0, seed=0)
        m = stb.Mesh(ctx, me.vtx, me.tets)
        w = np.ones(me.nt)
        row = {"panels": me.nt}
        searches = [("tree_nmin%d" % k, stb.default_params(lit_search=stb.STB_LIT_TREE, n_min=k))
                    for k in (8, 32, 64)]
        searches.append(("flat", stb.default_params(lit_search=stb.STB_LIT_FLAT)))
        for key, p in searches:
            stb.potential_S(ctx, m, w, pts, p)
            ts, tt = [], []
            for _ in range(reps):
                stb.potential_S(ctx, m, w, pts, p)
                ts.append(ctx.timings()["cull_ms"])
                tt.append(ctx.timings()["total_ms"])
            wk, ls = ctx.work(), ctx.lit_search()
            row[key] = {"cull_us_per_point": 1e3 * float(np.median(ts)) / npts,
                        "potential_us_per_point": 1e3 * float(np.median(tt)) / npts,
                        "leaf_panels_per_point": ls["leaf_panels"] / npts,
                        "candidates_per_point": wk["apex_pairs"] / npts,
                        "lit_per_point": wk["lit_pairs"] / npts}
        rows.append(row)
        m.close()
    n = np.array([r["panels"] for r in rows], dtype=np.float64)
    slopes = {k: float(np.polyfit(np.log(n[1:]), np.log([r[k]["cull_us_per_point"] for r in rows[1:]]), 1)[0])
              for k in rows[0] if k != "panels"}
    return {"points": npts, "meshes": rows, "slope_in_log_N": slopes,
            "note": "ball T=5, points at t=T uniform in the unit ball; cull phase only"}


def double_layer_leg(ctx, stb, mesh, npts, reps=3):
    """The retarded double-layer potential (eq. dlp) of a V_h^1 density with
    N(0,1) vertex values (seed 9) at the step's shell points, beside the
    single layer's potential at the same points; median of reps runs after
    one warm-up."""
    import numpy as np
    import torch
    from paper_2103_16841_amd import inputs
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    m.set_normals(mesh.outward_normals())
    v = inputs.density_normal(mesh.nv, seed=9)
    w = inputs.density_normal(mesh.nt, seed=5)
    pts = inputs.shell_points(npts, mesh.T, seed=4)
    res = {}
    for name, fn, dens in (("double_layer", stb.potential_D, v), ("single_layer", stb.potential_S, w)):
        fn(ctx, m, dens, pts)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(ctx, m, dens, pts)
            ts.append((time.perf_counter() - t0) * 1e3)
        res[name + "_ms"] = float(np.median(ts))
        res[name + "_candidates"] = ctx.work()["apex_pairs"]
    m.close()
    res["points"] = npts
    res["candidate_pairs_per_s"] = res["double_layer_candidates"] / (res["double_layer_ms"] * 1e-3)
    res["note"] = "host-to-device copies of points and densities included in both timings"
    return res


def direct_leg(ctx, stb):
    """The direct method (eq. df_dir) on the exterior of the unit sphere
    (icosphere level 2 x 16 slabs, T = 4) for the spherical wave
    mu(t - |x - y_S|) / |x - y_S|, mu(t) = t^3 e^-t, y_S = (-0.1, -0.2, -0.3):
    the L2 projection Q_h^1 g of the data, the right-hand side
    -1/2 b_I(Q g) + b_K(Q g), GMRES for the Neumann trace, Kirchhoff's
    formula u_h = D Q g - S w_h at three outside points at t = T."""
    import numpy as np
    import torch
    from paper_2103_16841_amd import inputs
    ys = np.array([-0.1, -0.2, -0.3])

    def mu(t, d=False):
        tp = np.maximum(t, 0.0)
        f = (3.0 * tp ** 2 - tp ** 3) if d else tp ** 3
        return np.where(t > 0.0, f * np.exp(-tp), 0.0)

    def u(p):
        r = np.linalg.norm(p[..., 1:] - ys, axis=-1)
        return mu(p[..., 0] - r) / r
    mesh = inputs.icosphere_mesh(level=2, S=16, T=4.0, jitter=0.0, seed=0)
    nrm = mesh.outward_normals()
    m = stb.Mesh(ctx, mesh.vtx, mesh.tets)
    m.set_normals(nrm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = stb.assemble_V(ctx, m)
    t1 = time.perf_counter()
    P, _ = stb.l2_points(ctx, m)
    g, cg_steps = stb.project_V1(ctx, m, u(P), mesh.nv)
    t15 = time.perf_counter()
    b = stb.dl_energetic(ctx, m, g, c_id=-0.5)
    t2 = time.perf_counter()
    x, its, rr = stb.solve_gmres(ctx, A, b, restart=100, maxit=20000, rtol=1e-10)
    t3 = time.perf_counter()
    cen = mesh.vtx[mesh.tets].mean(axis=1)
    y = cen[:, 1:]
    r = np.linalg.norm(y - ys, axis=1)
    tr = cen[:, 0] - r
    dn = np.einsum("ij,ij->i", ((-mu(tr, True) / r - mu(tr) / (r * r))[:, None] * (y - ys) / r[:, None]), nrm)
    far = np.array([[4.0, 1.5, 0.0, 0.3], [4.0, 0.2, -1.6, 0.0], [4.0, -1.2, 0.9, -0.6]])
    uh = stb.potential_D(ctx, m, g, far) - stb.potential_S(ctx, m, x, far)
    A.close()
    m.close()
    return {"mesh": "icosphere level 2 x 16 slabs, T=4 (N=%d)" % mesh.nt, "assemble_ms": (t1 - t0) * 1e3,
            "projection_ms": (t15 - t1) * 1e3, "projection_cg_steps": cg_steps,
            "rhs_ms": (t2 - t15) * 1e3, "gmres_ms": (t3 - t2) * 1e3, "products": its, "relres": rr,
            "neumann_rel_l2_error": float(np.linalg.norm(x - dn) / np.linalg.norm(dn)),
            "field_rel_error_max": float(np.max(np.abs(uh - u(far)) / np.abs(u(far))))}


def mixed_leg(args, ctx, stb, step, paramsmx, vtx_d, tet_d, nv, nt, rec):
    """The same step with the mixed-precision assembly; its entries compared
    with the FP64 assembly's (which match the oracle to 1e-10)."""
    import numpy as np
    import torch
    causal64 = rec["causal"]
    m = stb.Mesh.from_device(ctx, vtx_d.data_ptr(), nv, tet_d.data_ptr(), nt)
    A64 = stb.assemble_V(ctx, m)
    _, _, v64 = A64.export()
    A64.close()
    Amx = stb.assemble_V(ctx, m, paramsmx)
    _, _, vmx = Amx.export()
    Amx.close()
    # the mixed path with no far pairs: every node in FP64, outer points per
    # panel instead of per shared face -- a second FP64 evaluation of every
    # entry, whose distance from the first is the rounding noise of FP64
    # itself (large only where an entry's outer-point terms cancel)
    App = stb.assemble_V(ctx, m, stb.default_params(prec=stb.STB_MIXED, eta_far=1e300))
    _, _, vpp = App.export()
    App.close()
    m.close()
    # the stores hold the same causal pairs in the same order
    same = v64.shape == vmx.shape == vpp.shape
    if same:
        err = np.abs(vmx - vpp) / np.abs(vpp)        # against FP64 through the same outer points
        err_sf = np.abs(vmx - v64) / np.abs(v64)     # against the shared-face FP64 assembly
        noise = np.abs(vpp - v64) / np.abs(v64)      # the two FP64 assemblies
        above = int(np.count_nonzero(err > 1e-6))
        identical = int(np.count_nonzero(vmx == vpp))
    else:
        err = err_sf = noise = np.array([np.inf])
        above, identical = -1, -1
    zeros_ok = bool(same and np.all(vmx != 0.0))
    del v64, vmx, vpp
    acc = {}
    for _ in range(args.warmup):
        step(False, paramsmx, acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True, paramsmx, acc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    assert rec["causal"] == causal64
    kern = {k: v[0] / args.steps for k, v in acc.items() if v[1]}
    return {
        "value": causal64 / (ms * 1e-3), "unit": "causal element-pairs/s", "ms_per_step": ms,
        "max_rel_err_vs_fp64": float(err.max()),
        "err": "max over every causal entry of |A_mixed - A_fp64| / |A_fp64| (no floor), A_fp64 "
               "the FP64 assembly through the same per-panel outer points",
        "entries_above_1e-6": above,
        "entries_equal_to_fp64": identical,
        "max_rel_err_vs_fp64_shared_faces": float(err_sf.max()),
        "max_rel_diff_fp64_per_panel_vs_shared_faces": float(noise.max()),
        "same_causal_pairs": zeros_ok, "eta_far": paramsmx.eta_far,
        "kernel_ms_per_step": kern,
        "fp32_node_evals": acc.get("nodes_fp32", [0, 0, 0])[2] // args.steps,
        "entries_recomputed_fp64": acc.get("mixed_restore", [0, 0, 0])[2] // args.steps,
    }


def batch_leg(args, stb):
    """64 independent meshes (icosphere levels 0-3 x 8-64 slabs, T = 4,
    jitter +-0.2 dt, seed 3), each assembled (FP64, every causal pair, into
    its causal-only store) and applied to 16 right-hand sides on the FP32
    matrix cores; --batch-group meshes per call of the batched entry point,
    in HBM-budgeted waves.  One pass, timed from the first call to the last
    product (the launch-shape autotuner runs before, on the largest mesh)."""
    import numpy as np
    import torch
    from paper_2103_16841_amd import inputs

    dev = torch.device("cuda:0")
    mix = inputs.batch_mix(count=args.batch_count, seed=3)
    print("batch: %d meshes, %d panels" % (len(mix), sum(m.nt for m in mix)), file=sys.stderr,
          flush=True)
    ctx = stb.Context(0)
    meshes = [stb.Mesh(ctx, m.vtx, m.tets) for m in mix]
    W = [torch.from_numpy(np.random.default_rng(100 + k).standard_normal((m.nt, 16))).to(dev)
         for k, m in enumerate(mix)]
    Y = [torch.zeros_like(w) for w in W]
    big = max(range(len(mix)), key=lambda k: mix[k].nt)
    t_tune = time.perf_counter()
    blocks, per_cu = stb.autotune(ctx, meshes[big])
    t_tune = time.perf_counter() - t_tune
    print("tuned on mesh %d: blocks %s per CU %s" % (big, blocks, per_cu), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    causal = np.zeros(len(mix), dtype=np.int64)
    kt_acc, ev_acc, work = {}, {}, np.zeros(4, dtype=np.int64)
    t0 = time.perf_counter()
    g = args.batch_group
    for k0 in range(0, len(mix), g):
        c = np.zeros(min(g, len(mix) - k0), dtype=np.int64)
        stb.batch_assemble(ctx, meshes[k0:k0 + g], keep=False,
                           W_ptrs=[w.data_ptr() for w in W[k0:k0 + g]],
                           Y_ptrs=[y.data_ptr() for y in Y[k0:k0 + g]], causal=c)
        causal[k0:k0 + len(c)] = c
        for kk, (ms_k, n_k, u_k) in ctx.kernel_times().items():
            a = kt_acc.setdefault(kk, [0.0, 0, 0])
            a[0] += ms_k; a[1] += n_k; a[2] += u_k
        for kk, v in ctx.path_counts().items():
            ev_acc[kk] = ev_acc.get(kk, 0) + v
        wk = ctx.work()
        work += np.array([wk["L_evals"], wk["lit_pairs"], wk["apex_pairs"], wk["pieces"]])
        print("meshes %d..%d done, %.1f s, causal pairs so far %d" %
              (k0, k0 + len(c) - 1, time.perf_counter() - t0, causal.sum()), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ysum = float(sum(float(y.abs().sum()) for y in Y))
    ctx.close()
    k_ms, k_n, k_units = kt_acc.get("nodes_fp64", [0.0, 0, 0])
    avg_ms = k_ms / max(k_n, 1)
    achieved = k_units * C_NODE_FLOP / max(k_n, 1) / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    asm_flop = float(work[1]) * C_SETUP_FLOP + float(work[0]) * C_NODE_FLOP
    return {
        "value": float(causal.sum()) / dt, "unit": "causal element-pairs/s", "seconds": dt,
        "causal_pairs": int(causal.sum()), "meshes": len(mix), "panels": int(sum(m.nt for m in mix)),
        "largest_mesh": int(max(m.nt for m in mix)), "meshes_per_call": g,
        "autotune_s": t_tune, "tuned_blocks": blocks, "tuned_per_cu": per_cu,
        "workload": "%d icosphere meshes (levels 0-3 x 8-64 slabs, T=4, jitter +-0.2dt, seed 3), "
                    "each assembled (FP64, causal-only store) and applied to 16 RHS on the FP32 "
                    "matrix cores" % len(mix),
        "kernel_ms": {k: v[0] for k, v in kt_acc.items() if v[1]},
        "node_stage": {"kernel": "FP64 node stage", "achieved_tflops": achieved,
                       "frac": achieved / (FP64_VECTOR_PEAK / 1e12), "avg_launch_ms": avg_ms,
                       "launches": k_n, "path_counts": ev_acc},
        "assembly_tflops": asm_flop / dt / 1e12,
        "assembly_frac": asm_flop / dt / FP64_VECTOR_PEAK,
        "products_abs_sum": ysum,
    }


def batch_main(args):
    """The batched workload alone, as the main line."""
    import torch
    from paper_2103_16841_amd import stb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    b = batch_leg(args, stb)
    out = {
        "metric": METRIC, "value": b["value"], "unit": "causal element-pairs/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": b["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch: " + b["workload"], "causal_pairs": b["causal_pairs"]},
        "batch": b,
    }
    print(json.dumps(out), flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus %d refused); sharding across GPUs is "
              "a design, not built" % args.gpus, file=sys.stderr)
        return 2
    if args.workload == "batch":
        return batch_main(args)
    import numpy as np
    import torch
    from paper_2103_16841_amd import inputs, stb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    mesh = inputs.icosphere_mesh(level=2, S=32, T=4.0, jitter=0.2, seed=2)
    nt, nv = mesh.nt, mesh.nv
    vtx_d = torch.from_numpy(mesh.vtx).to(dev)
    tet_d = torch.from_numpy(mesh.tets.astype(np.int32)).to(dev)
    w_d = torch.from_numpy(inputs.density_normal(nt, seed=0)).to(dev)
    W_d = torch.from_numpy(np.random.default_rng(1).standard_normal((nt, 16))).to(dev)
    pts_d = torch.from_numpy(inputs.shell_points(args.points, mesh.T, seed=4)).to(dev)
    wp_d = torch.from_numpy(inputs.density_normal(nt, seed=5)).to(dev)
    y_d = torch.empty(nt, dtype=torch.float64, device=dev)
    Y_d = torch.empty((nt, 16), dtype=torch.float64, device=dev)
    u_d = torch.empty(args.points, dtype=torch.float64, device=dev)
    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    ctx = stb.Context(0)
    rec = {}

    kt_acc, ev_acc, asm_ms = {}, {}, []
    params64 = stb.default_params()
    paramsmx = stb.default_params(prec=stb.STB_MIXED)

    def step(timed, params=params64, acc=kt_acc):
        m = stb.Mesh.from_device(ctx, vtx_d.data_ptr(), nv, tet_d.data_ptr(), nt)
        A = stb.assemble_V(ctx, m, params)
        rec["timings"] = ctx.timings()
        rec["work"] = ctx.work()
        rec["causal"] = A.n_causal
        rec["stored"] = A.n_stored
        if timed:
            if acc is kt_acc:
                asm_ms.append(rec["timings"]["total_ms"])
            for k, (ms_k, n_k, u_k) in ctx.kernel_times().items():
                a = acc.setdefault(k, [0.0, 0, 0])
                a[0] += ms_k; a[1] += n_k; a[2] += u_k
            if acc is kt_acc:
                for k, v in ctx.path_counts().items():
                    ev_acc[k] = ev_acc.get(k, 0) + v
        A.apply_dev(w_d.data_ptr(), y_d.data_ptr(), 1)
        A.apply_dev(W_d.data_ptr(), Y_d.data_ptr(), 16)
        stb.potential_S_dev(ctx, m, wp_d.data_ptr(), args.points, pts_d.data_ptr(), u_d.data_ptr())
        A.close()
        m.close()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = rec["causal"] / (ms * 1e-3)
    # dominant kernel: the FP64 node stage; its launches were timed with HIP
    # events on the library's stream during the timed steps
    k_ms, k_n, k_units = kt_acc.get("nodes_fp64", [0.0, 0, 0])
    avg_ms = k_ms / max(k_n, 1)
    evals_per_launch = k_units / max(k_n, 1)
    achieved = evals_per_launch * C_NODE_FLOP / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    recipe_per_launch = node_flops(ev_acc) / max(k_n, 1)
    asm_med = float(np.median(asm_ms))
    work = rec["work"]
    asm_flop = work["lit_pairs"] * C_SETUP_FLOP + work["L_evals"] * C_NODE_FLOP
    asm_alg_bytes = 8 * rec["causal"] + 320 * nt
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "causal element-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "icosphere radius 1 level 2 (320 triangles) x 32 slabs, T=4, jitter "
                        "+-0.2dt seed 2, N=30720 panels: all causal pairs assembled, FP64 "
                        "matvec, 16-RHS FP32 MFMA apply, potential at %d shell points" % args.points,
            "n_panels": nt, "n_g": 16, "m_q": 3, "precision": "fp64",
            "causal_pairs": rec["causal"], "stored_entries": rec["stored"],
        },
        "phase_ms": rec["timings"],
        "assembly_ms_median": asm_med,
        "causal_pairs_per_s_assembly_only": rec["causal"] / (asm_med * 1e-3),
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt_acc.items() if v[1]},
        "roofline": {
            "bound": "alu",
            "kernel": "FP64 node stage (k_nodes_rec<1, true>, k_nodes_rec<1, false>, "
                      "k_nodes_rec<2, false>, k_nodes)",
            "achieved": achieved, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": achieved / (FP64_VECTOR_PEAK / 1e12), "traffic": K_NODES_TRAFFIC_BYTES,
            "flop_per_unit": "%g FLOP per evaluation of L(phi) (+ one sin/cos pair)" % C_NODE_FLOP,
            "L_evals_per_launch": evals_per_launch, "avg_launch_ms": avg_ms, "launches": k_n,
            "recipe_count": {"flop_per_L_by_path": FLOP_PER_L,
                             "node_evals_per_launch": {k: ev_acc.get(k, 0) / max(k_n, 1)
                                                       for k in FLOP_PER_L},
                             "tflops": recipe_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0},
            "ray_empty_pieces": ev_acc.get("ray_empty_pieces", 0) // args.steps,
            "assembly": {
                "flop": asm_flop,
                "flop_per_unit": "%g per lit (outer point, panel) pair + %g per evaluation of L"
                                 % (C_SETUP_FLOP, C_NODE_FLOP),
                "ms": asm_med, "tflops": asm_flop / (asm_med * 1e-3) / 1e12,
                "frac": asm_flop / (asm_med * 1e-3) / FP64_VECTOR_PEAK,
                "algorithmic_bytes": asm_alg_bytes,
                "algorithmic_bytes_unit": "8 B per causal pair + 320 B per panel",
                "profiled_bytes": ASSEMBLY_TRAFFIC_BYTES,
            },
            "work": work,
        },
    }
    if not args.no_solve:
        out["solve"] = solve_leg(ctx, stb, mesh)
    if not args.no_dl:
        out["double_layer"] = double_layer_leg(ctx, stb, mesh, args.points)
    if not args.no_litsearch:
        out["lit_search"] = lit_search_leg(ctx, stb)
    if args.direct:
        out["direct"] = direct_leg(ctx, stb)
    if not args.no_mixed:
        out["mixed"] = mixed_leg(args, ctx, stb, step, paramsmx, vtx_d, tet_d, nv, nt, rec)
    if not args.no_serving:
        out["serving"] = serving_leg(args, ctx, stb)
    ctx.close()
    if not args.no_batch:
        out["batch"] = batch_leg(args, stb)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, args.cpu_rows)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
