"""Benchmark: time-to-(1+eps) of the MWU solver on one MI355X, chosen form
(FP32 weights and search terms, FP64 totals, decisions and, where rounding
would grow, the direction) against the plain FP64 form, plus the HBM
throughput of the sparse product passes.

Headline workload (the largest configuration that fits one GPU): the densest
subgraph LP (the dual of Charikar's LP with D searched, Section 3 of the
paper) on a seeded R-MAT graph, scale 22, edge factor 16, a/b/c =
0.57/0.19/0.19, self-loops and duplicates removed, eps = 0.1: 64.2M edges,
128.3M variables.  A synthetic stand-in for the paper's Graph500 Kronecker
inputs.  A step is one full solve (outer search over D, every MWU iteration,
step searches, level-set bounds and certificates) with the graph already
resident in HBM.

The line also carries the same solve with the fastest measured setting
(warm-started search, probe reuse, dropping met covering rows), the
vertex-cover LP on R-MAT scale 20 and the batch of 512 bipartite-matching
LPs as extra keys (``--no-extra`` leaves the last two out), the
roofline of the dominant kernel (algorithmic bytes over its mean launch
duration, HIP events on the solver stream) and the plain FP64 CPU oracle
timed on a bounded sample of the same workload on one host core.

Prints one JSON line.
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-(1+eps) at eps=0.1 + A/A^T nnz/s (HBM GB/s), chosen vs plain FP64"
HBM_PEAK_GBPS = 8000.0
PASS_NAMES = {0: "row_pass", 1: "column_pass", 2: "forward_pass", 3: "search_pass_exp",
              4: "search_pass_bisect", 5: "search_pass_combined"}
VC_PASS_NAMES = {0: "transpose_pass", 1: "direction_pass", 2: "forward_pass", 3: "search_pass_exp",
                 4: "search_pass_bisect", 5: "search_pass_combined"}
DN_KERNELS = {0: "dn_row", 1: "dn_col", 2: "dn_fwd_v", 3: "dn_search"}
VC_KERNELS = {0: "vc_passA_k", 1: "vc_passB_k", 3: "vc_search_k"}
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def rmat_graph(scale, edge_factor, seed):
    import graphgen as gg
    return gg.cached(f"rmat{scale}_ef{edge_factor}_s{seed}", lambda: gg.rmat(scale, edge_factor, seed=seed))


def step_rule_of(mwu, args):
    return {"bin": mwu.STEP_BIN, "warm": mwu.STEP_BIN_WARM, "newton": mwu.STEP_NEWTON}[args.step_rule]


def timed_solves(s, steps, warmup, tag):
    """Solves timed with the result left on the device (x is not copied to
    the host: the inputs are resident and so is the answer)."""
    import torch
    walls, r = [], None
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = s.solve(want_x=False)
        w = time.perf_counter() - t
        if i >= warmup:
            walls.append(w)
        log(f"  {tag} solve {i}: {w:.4f}s obj={r.objective:.4f} [{r.lower:.4f}, {r.upper:.4f}] "
            f"status={r.status} iters={r.total_iterations} probes={r.probes} passes={r.search_passes} "
            f"evaluations={r.evaluations}")
    return walls, r


def pass_times(s, reps, param, warm_iters=0, last=0):
    """Average duration of each pass's main kernel (HIP events on the solver
    stream, state held), its algorithmic bytes and nonzeros, after warm_iters
    iterations of a probe at param.  Pass `last` (the dominant one) is timed
    last: every timing first forms one direction (a row, column and forward
    pass of its own), so only then are its held launches the last ones of its
    kernel, as the summaries under profiles/ assume."""
    out = {}
    s.probe_begin(param)
    if warm_iters:
        info = s.probe_run(warm_iters)
        log(f"  pass timing at iteration {info.iterations} of a probe at {param:.6g} (status {info.status})")
    for which in [w for w in (0, 1, 2, 3, 4, 5) if w != last] + [last]:
        us, by, nz = s.time_pass(which, reps)
        if by <= 0.0:       # a pass fused into another one (no kernel of its own)
            continue
        out[which] = {"us": us, "bytes": by, "nnz": nz, "GBps": by / us / 1e3,
                      "nnz_per_s": nz / (us * 1e-6) if nz else None}
    return out


def _shares(passes, r, kernels):
    """Each pass's time per iteration, the dominant one, and the pass index
    whose held launches stand for it (the combined pass for the search)."""
    spi = r.search_passes / max(1, r.total_iterations)
    extra = max(0.0, spi - 1.0)
    fallback_us = 0.5 * (passes[3]["us"] + passes[4]["us"])
    search_us = (passes[5]["us"] + extra * fallback_us) / (1.0 + extra)
    share = {k: passes[k]["us"] for k in (0, 1, 2) if k in passes and k in kernels}
    share[3] = spi * search_us
    dom = max(share, key=share.get)
    return share, dom, 5 if dom == 3 else dom


def dominant(passes, r, kernels, names, tag, workload):
    """The pass with the largest share of one iteration: one row pass, one
    column pass, one forward pass, and the search passes (the combined first
    pass, plus exponential-grid or bisection passes in the iterations the
    combined pass does not settle).  Its roofline is reported for its common
    launch (the combined pass for the search)."""
    from paper_2307_03307_amd import profiling
    share, dom, dom_pass = _shares(passes, r, kernels)
    kernel = kernels[dom]
    tname = "float" if tag == "f32" else "double"
    full = f"{kernel}<{tname}, false>" if kernel.endswith(("_fwd_v", "k_fwd")) else f"{kernel}<{tname}>"
    us, by = passes[dom_pass]["us"], passes[dom_pass]["bytes"]
    achieved = by / us / 1e3
    traffic = profiling.load_traffic(os.path.join(PROFILES, f"{kernel}_{workload}_{tag}_traffic.txt"), full)
    return {"bound": "hbm", "kernel": full,
            "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic, "avg_launch_us": us, "algorithmic_bytes": by, "pass": names[dom_pass],
            "share_of_iteration": share[dom] / sum(share.values()),
            "pass_share": {names[5 if k == 3 else k]: v / sum(share.values()) for k, v in share.items()}}


# ------------------------------------------------------------------ CPU oracle

def cpu_baseline_densest(g, param, gpu_iters, gpu_evals):
    """The plain FP64 oracle on one host core, on a bounded sample of the same
    workload: a probe set up with no iteration and one with one iteration of
    the standard step (no search) give the per-iteration cost of the passes;
    one iteration with Algorithm 3 adds its evaluations of the test.  The GPU solve's iteration
    and evaluation counts (the evaluations a one-at-a-time Algorithm 3 makes,
    counted on the device) scale the two costs."""
    import oracle
    oracle.build()
    t = time.perf_counter()
    O, W, keep = oracle.densest_matrices(g)
    build_s = time.perf_counter() - t
    sP = 1.0 / param

    def run(rule, iters):
        t = time.perf_counter()
        r = oracle.probe(O, sP, W, 1.0, 0.1, max_iter=iters, step_rule=rule)
        return time.perf_counter() - t, r

    t0, _ = run(oracle.STEP_STD, 0)
    t1, _ = run(oracle.STEP_STD, 1)
    tb, rb = run(oracle.STEP_BIN, 1)
    per_iter = max(t1 - t0, 1e-9)
    per_eval = max(tb - t1, 0.0) / max(1, rb.evaluations)
    est = per_iter * gpu_iters + per_eval * gpu_evals
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (plain single-threaded FP64 C, gcc -O2) on the same graph and LP at D = {param:.6g}: "
                       f"probes of 0 and 1 iterations with the standard step ({t0:.1f} s, {t1:.1f} s) and one "
                       f"iteration of Algorithm 3 ({tb:.1f} s, {rb.evaluations} evaluations); "
                       f"{per_iter:.2f} s per iteration x {gpu_iters} iterations + {per_eval:.2f} s per "
                       f"evaluation x {gpu_evals} evaluations of the GPU solve; explicit matrix build "
                       f"{build_s:.1f} s not counted"),
            "per_iteration_s": per_iter, "per_evaluation_s": per_eval, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count()}


def cpu_baseline_vcover(g, gpu_iters, gpu_evals, param):
    """As cpu_baseline_densest, for the vertex-cover LP."""
    import numpy as np
    import oracle
    oracle.build()
    C, keep = oracle.vertex_cover_matrix(g)
    n = C.cols
    ones = oracle.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))

    def run(rule, iters):
        t = time.perf_counter()
        r = oracle.probe(ones, 1.0 / param, C, 1.0, 0.1, max_iter=iters, step_rule=rule)
        return time.perf_counter() - t, r

    t1, _ = run(oracle.STEP_STD, 1)
    t2, _ = run(oracle.STEP_STD, 3)
    tb, rb = run(oracle.STEP_BIN, 1)
    per_iter = max(t2 - t1, 1e-9) / 2
    per_eval = max(tb - t1, 0.0) / max(1, rb.evaluations)
    est = per_iter * gpu_iters + per_eval * gpu_evals
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on the same graph at M = {param:.6g}: 1 and 3 standard-step iterations, one "
                       f"Algorithm 3 iteration ({rb.evaluations} evaluations); {per_iter:.3f} s per iteration x "
                       f"{gpu_iters} + {per_eval:.3f} s per evaluation x {gpu_evals}"),
            "per_iteration_s": per_iter, "per_evaluation_s": per_eval, "cpu_model": cpu_model()}


# ------------------------------------------------------------------ workloads

def run_densest(args, steps, warmup, with_cpu=True):
    """Densest subgraph (Charikar's dual, D searched): fused program, chosen
    form vs plain FP64.  No exact optimum exists at this size; a run counts
    when its bracket (level-set lower bound, rescaled feasible upper bound) is
    within 1 + eps."""
    import torch
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    t = time.perf_counter()
    g = rmat_graph(args.scale, args.edge_factor, 3)
    log(f"graph: {g.num_vertices} vertices, {g.num_edges} edges ({time.perf_counter() - t:.1f}s)")

    def run(precision, steps, warmup):
        t = time.perf_counter()
        s = mwu.densest_subgraph(g.num_vertices, g.u, g.v, precision=precision, step_rule=step_rule_of(mwu, args))
        create = time.perf_counter() - t
        walls, r = timed_solves(s, steps, warmup, f"densest precision={precision}")
        # one more solve returning x: the copy of the 2E doubles to the host
        t = time.perf_counter()
        rx = s.solve(want_x=True)
        x_host = time.perf_counter() - t - statistics.mean(walls)
        assert rx.total_iterations == r.total_iterations
        passes = pass_times(s, args.pass_reps, param=0.5 * (r.lower + r.upper), warm_iters=args.pass_warm_iters,
                            last=1)
        s.close()
        passes["x_to_host_s"] = x_host
        return create, walls, r, passes

    # the fastest measured setting beside the default one (solved first, so
    # that each form's held pass repetitions are the last launches of its
    # kernels in a profiled run): the warm-started
    # search (R19), probe-to-probe reuse (R21) and dropping met covering rows
    # (R22), in both forms (with it FP64 needs far fewer refinement passes)
    fast_flags = mwu._lib.FLAG_REUSE | mwu._lib.FLAG_DROP_SATISFIED
    fastest = {"step_rule": "warm", "flags": "reuse+drop"}
    for key, prec in (("chosen", mwu.MIXED_FP32_FP64), ("fp64", mwu.FP64)):
        with mwu.densest_subgraph(g.num_vertices, g.u, g.v, precision=prec,
                                  step_rule=mwu.STEP_BIN_WARM, flags=fast_flags) as s:
            wf, rf = timed_solves(s, 2, 1, f"densest warm start, reuse, drop, precision={prec}")
        fastest[key] = {"s": statistics.mean(wf), "certified": rf.certified, "bracket": [rf.lower, rf.upper],
                        "iterations": rf.total_iterations, "probes": rf.probes,
                        "search_passes": rf.search_passes, "evaluations": rf.evaluations}
    c32, w32, r32, p32 = run(mwu.MIXED_FP32_FP64, steps, warmup)
    c64, w64, r64, p64 = run(mwu.FP64, args.fp64_steps, 1 if args.fp64_steps > 1 else 0)
    t32, t64 = statistics.mean(w32), statistics.mean(w64)
    x_host32, x_host64 = p32.pop("x_to_host_s"), p64.pop("x_to_host_s")
    workload = f"rmat{args.scale}"
    out = {
        "metric": METRIC, "value": t32, "unit": "s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": 1000.0 * t32, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"densest subgraph LP (Charikar dual, D searched), R-MAT scale {args.scale}, "
                               f"edge factor {args.edge_factor}, a/b/c=0.57/0.19/0.19, seed 3, eps=0.1",
                   "vertices": g.num_vertices, "edges": g.num_edges, "variables": 2 * g.num_edges,
                   "form": "FP32 weights and search terms; FP64 x, d, rows, totals and decisions",
                   "step_rule": args.step_rule},
        "certified": r32.certified, "objective": r32.objective, "bracket": [r32.lower, r32.upper],
        "iterations": r32.total_iterations, "probes": r32.probes, "search_passes": r32.search_passes,
        "evaluations": r32.evaluations, "create_s": c32,
        "fp64_plain_s": t64, "fp64_steps": len(w64), "fp64_certified": r64.certified,
        "fp64_bracket": [r64.lower, r64.upper], "fp64_iterations": r64.total_iterations,
        "fp64_search_passes": r64.search_passes, "speedup_vs_fp64": t64 / t32,
        "x_to_host_s": x_host32, "x_to_host_s_fp64": x_host64, "fastest_setting": fastest,
        "passes": {PASS_NAMES[k]: v for k, v in p32.items()},
        "passes_fp64": {PASS_NAMES[k]: v for k, v in p64.items()},
        "roofline": dominant(p32, r32, DN_KERNELS, PASS_NAMES, "f32", workload),
        "roofline_fp64": dominant(p64, r64, DN_KERNELS, PASS_NAMES, "f64", workload),
    }
    out["A_nnz_per_s"] = p32[2]["nnz_per_s"] if 2 in p32 else None
    if with_cpu:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"] = cpu_baseline_densest(g, 0.5 * (r32.lower + r32.upper), r32.total_iterations,
                                                   r32.evaluations)
    return out


def run_passes_only(args):
    """Counter runs: the held pass timings of one precision at a fixed probe
    parameter, with no solve, then (``--copy-calib-mib``) the calibration
    copy.  Prints the pass timings as one JSON line."""
    import torch
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    prec = mwu.FP64 if args.precision == "fp64" else mwu.MIXED_FP32_FP64
    if args.workload == "densest":
        g = rmat_graph(args.scale, args.edge_factor, 3)
        s = mwu.densest_subgraph(g.num_vertices, g.u, g.v, precision=prec, step_rule=step_rule_of(mwu, args))
        passes = pass_times(s, args.pass_reps, args.pass_only, warm_iters=args.pass_warm_iters, last=1)
        names = PASS_NAMES
    elif args.workload == "domset":
        import graphgen as gg
        g = gg.cached("chunglu2m_g23_d10_s4", lambda: gg.chung_lu(2_000_000, 2.3, 10.0, seed=4))
        ptr, col = gg.adjacency_csr(g, with_identity=True)
        s = mwu.dominating_set(ptr, col, g.num_vertices, precision=prec, step_rule=step_rule_of(mwu, args))
        passes = pass_times(s, args.pass_reps, args.pass_only, warm_iters=600, last=1)
        names = PASS_NAMES
    else:
        g = rmat_graph(args.scale, args.edge_factor, 2)
        s = mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=prec, step_rule=step_rule_of(mwu, args))
        passes = pass_times(s, args.pass_reps, args.pass_only, warm_iters=600, last=0)
        names = VC_PASS_NAMES
    s.close()
    return {"workload": args.workload, "scale": args.scale, "param": args.pass_only, "precision": args.precision,
            "passes": {names[k]: v for k, v in passes.items()}}


def copy_calibration(mib):
    """A plain device copy of `mib` MiB (the counters' scale reference)."""
    import torch
    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def run_vcover(args, steps, warmup, scale=20, with_cpu=False):
    """Vertex cover LP (min 1^T x s.t. M^T x >= 1) via the implicit edge-list
    incidence on R-MAT scale 20: fused program with sparse passes."""
    import torch
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    t = time.perf_counter()
    g = rmat_graph(scale, args.edge_factor, 2)
    log(f"graph: {g.num_vertices} vertices, {g.num_edges} edges ({time.perf_counter() - t:.1f}s)")

    def run(precision, steps, warmup):
        t = time.perf_counter()
        s = mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision, step_rule=step_rule_of(mwu, args))
        create = time.perf_counter() - t
        walls, r = timed_solves(s, steps, warmup, f"vcover precision={precision}")
        # one iteration in, before any active list exists (full lists), then
        # 600 iterations in (the sparse phase, where most of a solve runs)
        full = pass_times(s, args.pass_reps, param=0.5 * (r.lower + r.upper), warm_iters=1, last=0)
        passes = pass_times(s, args.pass_reps, param=0.5 * (r.lower + r.upper), warm_iters=600, last=0)
        s.close()
        passes["full_list"] = full
        return create, walls, r, passes

    c32, w32, r32, p32 = run(mwu.MIXED_FP32_FP64, steps, warmup)
    c64, w64, r64, p64 = run(mwu.FP64, max(1, steps // 2), 1)
    f32, f64 = p32.pop("full_list"), p64.pop("full_list")
    t32, t64 = statistics.mean(w32), statistics.mean(w64)
    out = {
        "workload": f"vertex cover LP, R-MAT scale {scale}, edge factor {args.edge_factor}, seed 2, eps=0.1",
        "vertices": g.num_vertices, "edges": g.num_edges, "value": t32, "unit": "s", "steps": steps,
        "certified": r32.certified, "objective": r32.objective, "bracket": [r32.lower, r32.upper],
        "iterations": r32.total_iterations, "probes": r32.probes, "search_passes": r32.search_passes,
        "evaluations": r32.evaluations, "create_s": c32, "fp64_plain_s": t64, "fp64_certified": r64.certified,
        "fp64_iterations": r64.total_iterations, "speedup_vs_fp64": t64 / t32,
        "passes": {VC_PASS_NAMES[k]: v for k, v in p32.items()},
        "passes_fp64": {VC_PASS_NAMES[k]: v for k, v in p64.items()},
        "passes_full_list": {VC_PASS_NAMES[k]: v for k, v in f32.items()},
        "passes_full_list_fp64": {VC_PASS_NAMES[k]: v for k, v in f64.items()},
        "roofline": dominant(p32, r32, VC_KERNELS, VC_PASS_NAMES, "f32", f"rmat{scale}"),
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline_vcover(g, r32.total_iterations, r32.evaluations,
                                                  0.5 * (r32.lower + r32.upper))
    return out


GEN_KERNELS = {0: "k_row", 1: "k_col", 2: "k_fwd", 3: "k_search"}


def run_small(args, steps, warmup):
    """The small bipartite matching LP (2000 + 2000 vertices, 20,000 distinct
    uniform edges, seed 1; packing, max 1^T x s.t. M x <= 1): a solve here is
    bound by launch and finisher latency, not by HBM, so the figure is the
    time per MWU iteration next to the whole solve, in both forms, with the
    plain FP64 oracle's whole solve of the same LP timed beside it (the full
    workload: it finishes in seconds on one host core)."""
    import torch
    import graphgen as gg
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    g = gg.bipartite_uniform(2000, 2000, 20000, seed=1)
    out = {"workload": "bipartite matching LP, 2000 + 2000 vertices, 20,000 uniform edges, seed 1, eps=0.1",
           "vertices": g.num_vertices, "edges": g.num_edges}
    for tag, prec in (("", mwu.MIXED_FP32_FP64), ("fp64_", mwu.FP64)):
        with mwu.bmatch(g.num_vertices, g.u, g.v, precision=prec, step_rule=step_rule_of(mwu, args)) as s:
            walls, r = timed_solves(s, steps, warmup, f"small precision={prec}")
        t = statistics.mean(walls)
        out.update({f"{tag}s": t, f"{tag}certified": r.certified, f"{tag}bracket": [r.lower, r.upper],
                    f"{tag}iterations": r.total_iterations, f"{tag}probes": r.probes,
                    f"{tag}search_passes": r.search_passes,
                    f"{tag}us_per_iteration": 1e6 * t / max(1, r.total_iterations)})
    out["value"] = out.pop("s")
    out["unit"] = "s"
    out["steps"] = steps
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        M = oracle.incidence(g)
        rule = {"bin": oracle.STEP_BIN, "warm": oracle.STEP_BIN_WARM, "newton": oracle.STEP_NEWTON}[args.step_rule]
        reps, t = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t < 2.0:
            ro = oracle.solve_packing(M, step_rule=rule)
            reps += 1
        wall = (time.perf_counter() - t) / reps
        out["cpu_baseline"] = {
            "value": wall, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"the whole workload, mean of {reps} runs: the oracle's outer search on the same LP "
                       f"({ro.probes} probes, {ro.total_iterations} iterations, bracket "
                       f"[{ro.lower:.6g}, {ro.upper:.6g}])"),
            "us_per_iteration": 1e6 * wall / max(1, ro.total_iterations), "cpu_model": cpu_model()}
    return out


def cpu_baseline_domset(g, gpu_iters, gpu_evals, param):
    """As cpu_baseline_vcover, for the dominating-set LP (I + A)x >= 1."""
    import numpy as np
    import oracle
    oracle.build()
    C = oracle.dominating_set_matrix(g)
    n = C.cols
    ones = oracle.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))

    def run(rule, iters):
        t = time.perf_counter()
        r = oracle.probe(ones, 1.0 / param, C, 1.0, 0.1, max_iter=iters, step_rule=rule)
        return time.perf_counter() - t, r

    t1, _ = run(oracle.STEP_STD, 1)
    t2, _ = run(oracle.STEP_STD, 3)
    tb, rb = run(oracle.STEP_BIN, 1)
    per_iter = max(t2 - t1, 1e-9) / 2
    per_eval = max(tb - t1, 0.0) / max(1, rb.evaluations)
    return {"value": per_iter * gpu_iters + per_eval * gpu_evals, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on the same graph at M = {param:.6g}: 1 and 3 standard-step iterations, one "
                       f"Algorithm 3 iteration ({rb.evaluations} evaluations); {per_iter:.3f} s per iteration x "
                       f"{gpu_iters} + {per_eval:.3f} s per evaluation x {gpu_evals}"),
            "per_iteration_s": per_iter, "per_evaluation_s": per_eval, "cpu_model": cpu_model()}


def run_domset(args, steps, warmup):
    """Dominating set LP ((I + A)x >= 1) on a Chung-Lu power-law graph (2M
    vertices, exponent 2.3, mean degree 10, seed 4; 21.6M nonzeros): the
    generic CSR engine with its LDS-staged long rows, whole solves in both
    forms, without and with probe reuse, the held pass timings 600 iterations
    into a probe and the roofline of the dominant kernel."""
    import torch
    import graphgen as gg
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    t = time.perf_counter()
    g = gg.cached("chunglu2m_g23_d10_s4", lambda: gg.chung_lu(2_000_000, 2.3, 10.0, seed=4))
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    log(f"graph: {g.num_vertices} vertices, {g.num_edges} edges, {len(col)} nonzeros "
        f"({time.perf_counter() - t:.1f}s)")

    def run(precision, flags, steps, warmup, passes=False):
        t = time.perf_counter()
        s = mwu.dominating_set(ptr, col, g.num_vertices, precision=precision, flags=flags,
                               step_rule=step_rule_of(mwu, args))
        create = time.perf_counter() - t
        walls, r = timed_solves(s, steps, warmup, f"domset precision={precision} flags={flags}")
        p = None
        if passes:
            # timed twice: the dominant pass goes last the second time, so that
            # its held launches are the last ones of its kernel
            param = 0.5 * (r.lower + r.upper)
            p = pass_times(s, args.pass_reps, param, warm_iters=600, last=1)
            dom_pass = _shares(p, r, GEN_KERNELS)[2]
            p = pass_times(s, args.pass_reps, param, warm_iters=600, last=dom_pass)
        s.close()
        return create, statistics.mean(walls), r, p

    # the reuse run first: the chosen form's held launches are then the last
    # of their kernels in the process
    _, tr32, rr32, _ = run(mwu.MIXED_FP32_FP64, mwu._lib.FLAG_REUSE, 2, 1)
    c32, t32, r32, p32 = run(mwu.MIXED_FP32_FP64, 0, steps, warmup, passes=True)
    _, t64, r64, p64 = run(mwu.FP64, 0, 1, 0, passes=True)
    out = {
        "workload": "dominating set LP (I + A)x >= 1, Chung-Lu power law, 2M vertices, exponent 2.3, "
                    "mean degree 10, seed 4, eps=0.1",
        "vertices": g.num_vertices, "edges": g.num_edges, "nonzeros": int(len(col)),
        "value": t32, "unit": "s", "steps": steps, "certified": r32.certified, "objective": r32.objective,
        "bracket": [r32.lower, r32.upper], "iterations": r32.total_iterations, "probes": r32.probes,
        "search_passes": r32.search_passes, "evaluations": r32.evaluations, "create_s": c32,
        "fp64_plain_s": t64, "fp64_certified": r64.certified, "fp64_iterations": r64.total_iterations,
        "speedup_vs_fp64": t64 / t32,
        "reuse_s": tr32, "reuse_certified": rr32.certified, "reuse_iterations": rr32.total_iterations,
        "reuse_probes": rr32.probes,
        "passes": {PASS_NAMES[k]: v for k, v in p32.items()},
        "passes_fp64": {PASS_NAMES[k]: v for k, v in p64.items()},
        "roofline": dominant(p32, r32, GEN_KERNELS, PASS_NAMES, "f32", "chunglu2m"),
        "roofline_fp64": dominant(p64, r64, GEN_KERNELS, PASS_NAMES, "f64", "chunglu2m"),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"] = cpu_baseline_domset(g, r32.total_iterations, r32.evaluations,
                                                  0.5 * (r32.lower + r32.upper))
    return out


def run_batched(args, steps, warmup):
    """Batched bipartite matching: 512 uneven instances (sides uniform in
    [1024, 65536], mean degree uniform in [4, 16]) solved together with the
    built-in layout, against the plain FP64 form of the same batch, a host
    loop of single-instance FP64 solves (timed on a sample of instances,
    scaled by edge count) and the layout a timed sweep picks."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_bipartite_matching
    import torch
    import graphgen as gg
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    t = time.perf_counter()
    gs = gg.batch_bipartite(args.instances)
    E = sum(g.num_edges for g in gs)
    V = sum(g.num_vertices for g in gs)
    log(f"batch: {len(gs)} instances, {V} vertices, {E} edges ({time.perf_counter() - t:.1f}s)")
    spec = [(g.num_vertices, g.u, g.v) for g in gs]

    def run(precision, steps, warmup, tune=False):
        t = time.perf_counter()
        b = mwu.BatchSolver(spec, precision=precision, tune=tune, step_rule=step_rule_of(mwu, args))
        create = time.perf_counter() - t
        layout = b.layout()
        log(f"  precision={precision} create {create:.2f}s layout {layout}")
        walls, res = [], None
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = b.solve()
            w = time.perf_counter() - t
            if i >= warmup:
                walls.append(w)
            cert = sum(r.certified for r in res)
            its = sum(r.total_iterations for r in res)
            log(f"  precision={precision} batch solve {i}: {w:.3f}s certified {cert}/{len(res)} "
                f"iterations {its} max probe count {max(r.probes for r in res)}")
        b.close()
        return create, walls, res, layout

    c32, w32, r32, lay32 = run(mwu.MIXED_FP32_FP64, steps, warmup)
    c64, w64, r64, lay64 = run(mwu.FP64, 1, 0)
    ctun, wtun, _, laytun = run(mwu.MIXED_FP32_FP64, 1, 0, tune=True)
    # exact optima of a sample (Hopcroft-Karp; the bipartite matching LP is integral)
    sample = list(range(0, len(gs), max(1, len(gs) // 8)))
    ok = 0
    for k in sample:
        g = gs[k]
        nl = g.n_left
        A = sp.csr_matrix((np.ones(g.num_edges), (g.u, g.v - nl)), shape=(nl, g.num_vertices - nl))
        nu = int((maximum_bipartite_matching(A, perm_type="column") >= 0).sum())
        r = r32[k]
        ok += r.certified and r.lower * (1 - 1e-12) <= nu <= r.upper * (1 + 1e-12)
    # host loop of single-instance FP64 solves on a sample, scaled by edges
    loop_n = min(args.loop_sample, len(gs))
    t = time.perf_counter()
    e_loop = 0
    for g in gs[:loop_n]:
        with mwu.bmatch(g.num_vertices, g.u, g.v, precision=mwu.FP64) as s1:
            s1.solve()
        e_loop += g.num_edges
    loop_s = (time.perf_counter() - t) * E / e_loop
    t32 = statistics.mean(w32)
    return {
        "workload": f"batched bipartite matching LPs: {len(gs)} instances, sides uniform in [1024, 65536], "
                    f"mean degree uniform in [4, 16], eps=0.1",
        "instances": len(gs), "vertices": V, "edges": E, "value": t32, "unit": "s", "steps": steps,
        "certified": sum(r.certified for r in r32), "exact_optimum_in_bracket": f"{ok}/{len(sample)}",
        "iterations": sum(r.total_iterations for r in r32), "create_s": c32,
        "layout": {k: lay32[k] for k in ("tile_edges", "tile_vertices", "workgroups_per_cu",
                                         "search_launches", "source", "candidates_timed")},
        "tuned_layout_s": wtun[0], "tuned_layout_create_s": ctun,
        "tuned_layout": {k: laytun[k] for k in ("tile_edges", "tile_vertices", "workgroups_per_cu",
                                                "search_launches", "source", "candidates_timed")},
        "fp64_batched_s": statistics.mean(w64), "fp64_batched_certified": sum(r.certified for r in r64),
        "fp64_loop_s": loop_s,
        "fp64_loop_sample": f"{loop_n} instances ({e_loop} edges) timed, scaled by total edges",
        "speedup_vs_fp64_batched": statistics.mean(w64) / t32, "speedup_vs_fp64_loop": loop_s / t32,
    }


def run_genmatch(args):
    """Generalized matching (the appendix's mixed feasibility LP l <= Mx <= u
    on a user-item graph; users 3..5 matches, items at most 200, no lower
    bound for items) on a seeded synthetic rating graph standing in for the
    Netflix data: one feasibility probe at lambda = 1, chosen form vs plain
    FP64, and the max violation max{0, max(Px) - 1, 1 - min(Cx)} along the
    chosen-form probe (the iterate before each checkpoint's last step)."""
    import numpy as np
    import scipy.sparse as sp
    import torch
    import graphgen as gg
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    t = time.perf_counter()
    users, items = args.gm_users, args.gm_items
    g = gg.cached(f"useritem_{users}_{items}_d10-60_z1_s31",
                  lambda: gg.user_item(users, items, 10, 60, 1.0, seed=31))
    V, E = g.num_vertices, g.num_edges
    log(f"user-item graph: {users} users, {items} items, {E} ratings ({time.perf_counter() - t:.1f}s)")
    lb_user, ub_user, cap = 3.0, 5.0, 200.0
    ub = np.where(np.arange(V) < users, ub_user, cap)
    lb = np.full(users, lb_user)
    e = np.arange(E)
    ptr = np.zeros(users + 1, np.int64)
    np.cumsum(np.bincount(g.u, minlength=users), out=ptr[1:])
    Ps = sp.csr_matrix((np.concatenate([1.0 / ub[g.u], 1.0 / ub[g.v]]),
                        (np.concatenate([g.u, g.v]), np.concatenate([e, e]))), shape=(V, E))
    Cs = sp.csr_matrix((np.full(E, 1.0 / lb_user), (g.u, e)), shape=(users, E))

    def make(precision, iters_per_launch=0):
        return mwu.Solver(mwu.MIXED, P=mwu.incidence(V, g.u, g.v),
                          C=mwu.csr_matrix(ptr, e.astype(np.int32), shape=(users, E)),
                          b_P=ub, b_C=lb, fixed_lambda=1.0, precision=precision,
                          step_rule=step_rule_of(mwu, args), iters_per_launch=iters_per_launch)

    def run(precision, steps, warmup):
        walls, r = [], None
        with make(precision) as s:
            for i in range(warmup + steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = s.solve()
                w = time.perf_counter() - t
                if i >= warmup:
                    walls.append(w)
                log(f"  precision={precision} genmatch solve {i}: {w:.4f}s status={r.status} "
                    f"iters={r.total_iterations} passes={r.search_passes} max violation {r.max_violation:.3g}")
        return walls, r

    w32, r32 = run(mwu.MIXED_FP32_FP64, args.steps, args.warmup)
    w64, r64 = run(mwu.FP64, 1, 0)
    curve = []   # (iterations, max violation), in steps of 2 iterations (a graph launch of 2)
    with make(mwu.MIXED_FP32_FP64, iters_per_launch=2) as s:
        n = s.sizes().n
        s.probe_begin(1.0)
        while True:
            info = s.probe_run(2)
            x = s.probe_read("x", n)
            viol = max(0.0, (Ps @ x).max() - 1.0, 1.0 - (Cs @ x).min())
            curve.append([int(info.iterations), float(viol)])
            if info.status != 0 or info.iterations >= 5000:
                break
    t32 = statistics.mean(w32)
    return {
        "metric": "time-to-feasibility of one generalized-matching probe, chosen vs plain FP64",
        "value": t32, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * t32, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"generalized matching l <= Mx <= u, synthetic user-item graph: {users} users "
                               f"rating 10..60 items each of {items} (popularity ~ rank^-1), users 3..5, "
                               f"items <= 200, eps=0.1", "vertices": V, "edges": E,
                   "step_rule": args.step_rule},
        "certified": r32.certified, "iterations": r32.total_iterations, "max_violation": r32.max_violation,
        "fp64_s": statistics.mean(w64), "fp64_iterations": r64.total_iterations,
        "fp64_max_violation": r64.max_violation, "speedup_vs_fp64": statistics.mean(w64) / t32,
        "max_violation_curve": curve,
    }


def run_steprules(args):
    """Step rules, probe-to-probe reuse (MWU_FLAG_REUSE) and dropping satisfied
    covering rows (MWU_FLAG_DROP_SATISFIED) compared on whole solves, chosen
    form: Algorithm 3 from 1 (bin), Algorithm 3 from the previous step (warm)
    and Newton's method (newton, Section 4.2), each without and with reuse,
    and the drop with two of them, on the vertex cover (R-MAT 20), densest subgraph
    (R-MAT 22) and dominating set (Chung-Lu, 2M vertices) workloads: time,
    probes, iterations, search passes (launches of the search kernel) and
    tests of the step (evaluations), with their per-iteration rates."""
    import torch
    import graphgen as gg
    import paper_2307_03307_amd as mwu
    assert torch.cuda.is_available(), "needs an MI355X"
    g2 = rmat_graph(20, args.edge_factor, 2)
    g3 = rmat_graph(22, args.edge_factor, 3)
    g4 = gg.cached("chunglu2m_g23_d10_s4", lambda: gg.chung_lu(2_000_000, 2.3, 10.0, seed=4))
    ptr4, col4 = gg.adjacency_csr(g4, with_identity=True)
    makers = {
        "vcover_rmat20": lambda **k: mwu.vertex_cover(g2.num_vertices, g2.u, g2.v, **k),
        "densest_rmat22": lambda **k: mwu.densest_subgraph(g3.num_vertices, g3.u, g3.v, **k),
        "domset_chunglu2m": lambda **k: mwu.dominating_set(ptr4, col4, g4.num_vertices, **k),
    }
    out = {"metric": "time-to-(1+eps) by step rule, probe-to-probe reuse and dropping met rows", "unit": "s",
           "runs": {}}
    rules = (("bin", mwu.STEP_BIN), ("warm", mwu.STEP_BIN_WARM), ("newton", mwu.STEP_NEWTON))
    F_REUSE, F_DROP = mwu._lib.FLAG_REUSE, mwu._lib.FLAG_DROP_SATISFIED
    # every rule with and without reuse; dropping satisfied covering rows
    # with Algorithm 3 fresh and with the warm start and reuse
    configs = [(rn, r, f) for rn, r in rules for f in (0, F_REUSE)]
    configs += [("bin", mwu.STEP_BIN, F_DROP), ("warm", mwu.STEP_BIN_WARM, F_REUSE | F_DROP)]
    for name, make in makers.items():
        for rule_name, rule, flags in configs:
            tag = ("reuse" if flags & F_REUSE else "fresh") + ("+drop" if flags & F_DROP else "")
            s = make(precision=mwu.MIXED_FP32_FP64, step_rule=rule, flags=flags)
            walls, r = timed_solves(s, 2, 1, f"{name} {rule_name} {tag}")
            s.close()
            it = max(1, r.total_iterations)
            out["runs"][f"{name}/{rule_name}/{tag}"] = {
                "s": statistics.mean(walls), "certified": r.certified, "bracket": [r.lower, r.upper],
                "probes": r.probes, "iterations": r.total_iterations, "search_passes": r.search_passes,
                "evaluations": r.evaluations, "passes_per_iteration": r.search_passes / it,
                "evaluations_per_iteration": r.evaluations / it}
    return out


def headline(args, d, workload):
    """Wrap a workload record in the fields of the one-line bench contract."""
    out = {"metric": METRIC, "value": d["value"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1000.0 * d["value"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": workload, "step_rule": args.step_rule}}
    out.update({k: v for k, v in d.items() if k not in ("value", "unit", "steps", "workload")})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["densest", "vcover", "batched", "genmatch", "steprules", "small",
                                           "domset"],
                    default="densest",
                    help="densest: the headline R-MAT scale 22 densest subgraph (default); vcover: R-MAT "
                         "vertex cover; batched: 512 matching LPs; genmatch: generalized matching; "
                         "steprules: step rules and probe reuse compared on three workloads; small: the "
                         "2000 + 2000 matching LP (time per iteration); domset: dominating set on a 2M-vertex "
                         "power-law graph (generic engine)")
    ap.add_argument("--scale", type=int, default=None, help="R-MAT scale (default 22 densest, 20 vcover)")
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: leave out the vertex-cover and batched records")
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed solves of the plain FP64 form")
    ap.add_argument("--pass-reps", type=int, default=50)
    ap.add_argument("--pass-warm-iters", type=int, default=48,
                    help="densest: iterations of a probe at the middle of the final bracket before the "
                         "passes are timed")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--gm-users", type=int, default=200000)
    ap.add_argument("--gm-items", type=int, default=20000)
    ap.add_argument("--loop-sample", type=int, default=16)
    ap.add_argument("--pass-only", type=float, default=None,
                    help="counter runs: time the passes of a probe at this parameter (densest D, vcover or "
                         "domset M) "
                         "and solve nothing")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed", help="with --pass-only")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="end with a plain device copy of this many MiB (scale of the HBM counters)")
    ap.add_argument("--step-rule", choices=["bin", "warm", "newton"], default="bin",
                    help="bin: Algorithm 3 from 1 in every iteration; warm: started at the previous step; "
                         "newton: Newton's method from the previous step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.scale is None:
        args.scale = 20 if args.workload == "vcover" else 22

    if args.pass_only is not None:
        out = run_passes_only(args)
    elif args.workload == "densest":
        out = run_densest(args, args.steps, args.warmup, with_cpu=not args.no_cpu_baseline)
        if not args.no_extra:
            out["vcover_rmat20"] = run_vcover(args, 3, 1)
            out["batched_512"] = run_batched(args, 2, 1)
    elif args.workload == "vcover":
        d = run_vcover(args, args.steps, args.warmup, scale=args.scale, with_cpu=not args.no_cpu_baseline)
        out = headline(args, d, d["workload"])
    elif args.workload == "batched":
        d = run_batched(args, args.steps, args.warmup)
        out = headline(args, d, d["workload"])
    elif args.workload == "steprules":
        out = run_steprules(args)
    elif args.workload == "small":
        d = run_small(args, args.steps, args.warmup)
        out = headline(args, d, d["workload"])
    elif args.workload == "domset":
        d = run_domset(args, args.steps, args.warmup)
        out = headline(args, d, d["workload"])
    else:
        out = run_genmatch(args)
    if args.copy_calib_mib:
        copy_calibration(args.copy_calib_mib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
