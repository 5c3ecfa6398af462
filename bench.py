"""Benchmark: Gravo MG setup + solve on one MI355X.

A step is one whole pass of the method on one system: build the hierarchy
(sampling, Voronoi cells, prolongation, Galerkin operators, colouring,
coarsest factorisation) and solve to 1e-8 relative residual with V-cycles.
The same steps are then timed with the solve done by conjugate gradients
preconditioned with the symmetric V-cycle in double and in float (the mixed
form), reported under "mixed_vs_fp64".
The workload is the 1024 x 1024 jittered torus (1,048,576 points) with the
cotan smoothing system (M + 1e-3 L) x = M b.  Inputs are resident in HBM
before the timed region starts.

Besides the headline the line carries: the whole step against the HBM
roofline (the algorithmic byte model below on the step's own level sizes),
the method's per-level statistics (coarsening ratio, fallback and
single-entry prolongation rows), the 2,000,000-point bumpy-sphere point
cloud (kNN graph) in the plain FP64 form and in the mixed form (float
V-cycles preconditioning double CG to 1e-10), the many-mesh batched form
against the plain double path on the same number of streams, and the CPU
oracle on one pinned host core.

Prints one JSON line (see the keys below).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, scaled by what the counters read
# for a plain device copy (profiles/k_gs_block_torus1024.md, profiles/k_gs_color_fine_torus1024.md);
# valid only for the kernel and layout sources they were taken on (sha256 prefix of solve.hip +
# rows.hpp + setup_solve.hip, which lays out the matrices and blocks the kernels read).
TRAFFIC = {"gs_finest": {"bytes_per_launch": 26110584, "src_sha256_16": "b297e82abd4cef97"},
           "gs_galerkin": {"bytes_per_launch": 12451111, "src_sha256_16": "b297e82abd4cef97"}}

KERNEL_NAMES = {"gs_finest": "k_gs_color_fine (one colour of a Gauss-Seidel sweep, level 0)",
                "residual_finest": "k_residual_norm (residual + norm partials, level 0)",
                "gs_galerkin": "k_gs_block (one block colour of a block-ordered Gauss-Seidel sweep, Galerkin levels above "
                               "the tail; k_gs_color<R> where a level has no block order)"}


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("solve.hip", "rows.hpp", "setup_solve.hip"):
        h.update(open(os.path.join(ROOT, "paper_2307_04886_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kind):
    rec = TRAFFIC.get(kind)
    if rec is None:
        return None
    return rec["bytes_per_launch"] if kernel_src_sha() == rec["src_sha256_16"] else None


# Algorithmic bytes of the method's data movement (each array read or written once per logical
# pass; 8 B per value, 4 B per index), on the actual level sizes.  n, z = nnz(A_l), p = nnz(P_l),
# m = undirected edges, nc = n_{l+1}.
def vcycle_bytes(lv, nu):
    """One V-cycle: nu sweeps, residual, restriction, prolongation + correction per level, the
    coarsest product with the dense inverse, and the level-0 residual of the convergence test."""
    tot = 0.0
    for l in range(len(lv) - 1):
        n, z, p, nc = lv[l]["n"], lv[l]["nnzA"], lv[l]["nnzP"], lv[l + 1]["n"]
        sweep = 12 * z + 28 * n
        tot += nu * sweep + sweep + (12 * p + 8 * n + 12 * nc) + (12 * p + 8 * nc + 16 * n)
    tot += 8 * lv[-1]["n"] ** 2
    return tot + 12 * lv[0]["nnzA"] + 28 * lv[0]["n"]


def setup_bytes(lv):
    """The build: inputs copied; per level the edge CSR, edge lengths and mean, the conflict test
    and sampling rounds (conflict entries counted as the edge CSR's 2m, a lower bound), one
    Voronoi relaxation pass, cells and shift, coarse edges, projection, P^T, the Galerkin
    product, colouring and the solve layouts; the coarsest factor and inverse."""
    tot = 0.0
    L = len(lv)
    for l, s in enumerate(lv):
        n, m, z = s["n"], s["m"], s["nnzA"]
        C = 2 * m
        if l == 0:
            tot += 24 * n + 8 * m + 12 * z
        tot += 16 * m + 4 * n + 28 * n + 24 * m
        if l + 1 < L:
            p, zc = s["nnzP"], lv[l + 1]["nnzA"]
            tot += 16 * m + (24 * m + 8 * n + 4 * C) + 2 * (4 * C + n) + (24 * m + 28 * n) + 36 * n
            tot += (8 * m + 8 * n) + 64 * n + 72 * n + (12 * z + 72 * n + 12 * zc) + 2 * (4 * z + 12 * n)
            tot += 24 * z + 24 * p
        else:
            tot += 24 * n * n
    return tot


def level_stats(h):
    """Per level: sizes, colours, coarsening ratio and the prolongation's fallback and
    single-entry rows (Sec. 4.4 reports a fallback rate of about 0.25%)."""
    import numpy as np
    out = []
    L = h.num_levels
    for l in range(L):
        s = h.sizes(l)
        row = {"n": s["n"], "edges": s["m"], "nnz_A": s["nnzA"], "colours": s["colors"],
               "block_order": s["blocks"], "kernel_shape": h.tuning(l)}
        if l + 1 < L:
            cnt = h.export(l, "p_cnt")
            row.update({"nnz_P": s["nnzP"], "coarse_points": s["samples"],
                        "coarsening_ratio": s["samples"] / s["n"],
                        "fallback_rows": s["fallback"], "fallback_pct": 100.0 * s["fallback"] / s["n"],
                        "single_entry_rows": int((cnt == 1).sum()),
                        "single_entry_pct": 100.0 * float((cnt == 1).mean())})
        out.append(row)
    return out


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "allowed_cores": len(os.sched_getaffinity(0)), "model": model}


def pinned(fn):
    """Runs fn() with the calling thread pinned to one allowed core (the equivalent of
    taskset -c <core>); returns (result, core)."""
    saved = os.sched_getaffinity(0)
    core = min(saved)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, saved)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_leg(args, dev, opt, forms=("f32", "grouped", "plain")):
    """Many meshes of uneven size with 8 right-hand sides each: every hierarchy built and every
    right-hand side solved to the same tolerance.  Forms: the grouped float-preconditioned CG
    (builds on 4 streams, then one CG over all hierarchies, every step one launch for all meshes);
    the same CG per mesh on the 4 streams; the plain double V-cycle solve of each right-hand side
    in turn on the same 4 streams."""
    import torch
    import synth
    from paper_2307_04886_amd.batch import solve_many
    batch = synth.config_batched()
    systems = []
    for bp, B in batch:
        t = [torch.from_numpy(a).to(dev) for a in (bp.points, bp.edges, bp.indptr, bp.indices, bp.data)]
        systems.append(tuple(t) + (torch.from_numpy(B).to(dev),))
    nsolves = sum(B.shape[0] for _, B in batch)
    progress("many-mesh workload generated")
    res = {"streams": args.batched_streams,
           "workload": f"{len(batch)} jittered tori and icospheres, {min(b.n for b, _ in batch)}"
                       f"-{max(b.n for b, _ in batch)} vertices ({sum(b.n for b, _ in batch)} in total),"
                       f" 8 right-hand sides each, (M + 1e-3 L), tol {args.tol}", "solves": nsolves}
    ns = args.batched_streams
    names = {"grouped": f"setup on {ns} streams + one float-preconditioned double CG over all hierarchies "
                        "(gmg_solve_pcg_grouped: each step one launch for all meshes, 8 right-hand sides each)",
             "f32": "setup + float-preconditioned double CG per mesh (gmg_solve_pcg_batched), 8 right-hand "
                    f"sides per launch, {ns} streams",
             "plain": f"setup + plain double V-cycle solve of each right-hand side in turn, the same {ns} streams"}
    for form in forms:
        kw = {"grouped": dict(precision="f32", form="grouped"), "f32": dict(precision="f32"),
              "plain": dict(max_iters=200, form="plain")}[form]
        solve_many(systems, streams=args.batched_streams, tol=args.tol, **kw)
        torch.cuda.synchronize()
        timing = {}
        t1 = time.perf_counter()
        r = solve_many(systems, streams=args.batched_streams, tol=args.tol, timing=timing, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        if any(st != 0 for _, _, st in r):
            raise RuntimeError(f"{form} many-mesh solve did not converge")
        progress(f"many-mesh {form}: {1e3 * dt:.1f} ms")
        rec = {"form": names[form], "value": nsolves / dt, "unit": "solves/s", "ms": 1e3 * dt}
        if timing:
            rec.update({"build_ms": 1e3 * timing["build_s"], "solve_ms": 1e3 * timing["solve_s"]})
        res[form] = rec
    main = "grouped" if "grouped" in res else "f32"
    if main in res:
        res.update({"value": res[main]["value"], "unit": "solves/s", "ms": res[main]["ms"], "main_form": main})
    for other in ("f32", "plain"):
        if other in res and main in res and other != main:
            res[f"vs_{other}"] = res[other]["ms"] / res[main]["ms"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-mesh batched measurement")
    ap.add_argument("--no-pointcloud", action="store_true", help="skip the 2M-point point-cloud measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the many-mesh batched measurement (for profiler runs)")
    ap.add_argument("--batched-streams", type=int, default=4,
                    help="streams (host threads) of the many-mesh builds and per-mesh solves (1: one thread, "
                         "for profiler runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the plain steps (and roofline passes): for profiler runs")
    ap.add_argument("--size", type=int, default=1024, help="torus grid size (default 1024)")
    ap.add_argument("--timer", default="auto", choices=["auto", "gs_finest", "gs_galerkin", "residual_finest", "none"],
                    help="kernel classes timed with HIP events for the roofline entries (auto: both Gauss-Seidel "
                         "classes, the one with the larger share of the step first)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run one plain 256 MiB device copy (reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method's single-mesh "
              "pipeline is measured per GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2307_04886_amd as g
    from paper_2307_04886_amd.binding import build_hierarchy, default_options, timer_start, timer_stop

    g.library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(args, dev, default_options(), forms=("f32", "grouped"))}), flush=True)
        return
    t0 = time.time()
    prob = synth.config_torus(args.size, args.size)
    gen_s = time.time() - t0
    pts = torch.from_numpy(prob.points).to(dev)
    edges = torch.from_numpy(prob.edges).to(dev)
    rp = torch.from_numpy(prob.indptr).to(dev)
    ci = torch.from_numpy(prob.indices).to(dev)
    va = torch.from_numpy(prob.data).to(dev)
    b = torch.from_numpy(prob.rhs).to(dev)
    x = torch.zeros_like(b)
    opt = default_options()
    stream = torch.cuda.current_stream()

    stats = {}

    def step(form="plain"):
        h = build_hierarchy(pts, edges, rp, ci, va, opt, stream)
        x.zero_()
        if form == "plain":
            _, info, st = h.solve(b, x, tol=args.tol, max_iters=100, stream=stream)
        else:
            _, info, st = h.solve_pcg(b, x, tol=args.tol, max_iters=100, precision=form[-3:], stream=stream)
        if st != 0:
            raise RuntimeError(f"{form} solve did not converge (status {st})")
        levels = h.num_levels
        if "levels" not in stats:
            stats["levels"] = level_stats(h)
            stats["sizes"] = [h.sizes(l) for l in range(levels)]
        h.free()
        return info, levels

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info, levels = infos[-1]
    ms = 1e3 * dt / args.steps
    progress(f"headline: {args.steps} steps, {ms:.2f} ms per step")
    x_plain = x.cpu().numpy()
    nu = opt.nu_pre + opt.nu_post
    sb, cb = setup_bytes(stats["sizes"]), vcycle_bytes(stats["sizes"], nu)
    step_b = sb + info.iterations * cb
    step_roofline = {"bound": "hbm", "what": "whole setup + solve step, algorithmic bytes",
                     "bytes": step_b, "setup_bytes": sb, "vcycle_bytes": cb, "v_cycles": info.iterations,
                     "achieved": step_b / (ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": step_b / (ms * 1e-3) / 8e12}

    # Roofline: the same K steps again, every launch of one kernel class timed with a pair of
    # HIP events recorded by the dispatch itself on the launch stream (instrumented launches are
    # issued outside the captured graph, so these passes are not the headline timing).
    def roofline_pass(kind):
        timer_start(kind, expected_launches=4000 * args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t1
        k_ms, k_launches, k_bytes = timer_stop()
        ach = k_bytes / (k_ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": KERNEL_NAMES[kind], "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                "frac": ach / 8000.0, "traffic": traffic_for(kind), "kernel_ms_per_step": k_ms / args.steps,
                "share_of_step": k_ms / (1e3 * pdt), "launches": k_launches,
                "avg_launch_us": 1e3 * k_ms / max(k_launches, 1), "bytes_per_launch": k_bytes / max(k_launches, 1)}

    kinds = {"auto": ["gs_galerkin", "gs_finest"], "none": []}.get(args.timer, [args.timer])
    lines = sorted([roofline_pass(k) for k in kinds], key=lambda r: -r["kernel_ms_per_step"])
    progress("roofline passes done")

    # the same workload solved by CG preconditioned with the symmetric V-cycle, in double and in
    # float (mixed precision): whole setup + solve per step, same tolerance
    forms = {}
    x_forms = {}
    for form in () if args.headline_only else ("pcg_f64", "pcg_f32"):
        for _ in range(max(1, args.warmup)):
            step(form)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        finfos = [step(form) for _ in range(args.steps)]
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t1
        fi = finfos[-1][0]
        x_forms[form] = x.cpu().numpy()
        forms[form] = {"value": args.steps / fdt, "ms_per_step": 1e3 * fdt / args.steps,
                       "iterations": fi.iterations, "rel_residual": fi.rel_residual,
                       "vs_plain_fp64": (args.steps / fdt) / (args.steps / dt)}

    # setup / solve split (separate, synchronised runs outside the timed regions)
    def split(form, reps=3):
        su, so = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            h = build_hierarchy(pts, edges, rp, ci, va, opt, stream)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            x.zero_()
            if form == "plain":
                h.solve(b, x, tol=args.tol, max_iters=100, stream=stream)
            else:
                h.solve_pcg(b, x, tol=args.tol, max_iters=100, precision=form[-3:], stream=stream)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            h.free()
            su.append(tb - ta)
            so.append(tc - tb)
        return {"setup_ms": 1e3 * float(np.median(su)), "solve_ms": 1e3 * float(np.median(so))}

    # the 2,000,000-point bumpy sphere (kNN k = 8, Gaussian graph Laplacian): plain FP64 to
    # 1e-8 and the mixed form (float V-cycles preconditioning double CG) to 1e-10, each a whole
    # setup + solve per step; errors against a plain FP64 solve to 1e-12 (the plain path's
    # iterates are bit-identical to the oracle's FP64 iterates)
    pointcloud = None
    if not args.no_pointcloud and not args.headline_only:
        t0 = time.time()
        pc = synth.config_bumpy_sphere()
        pc_gen = time.time() - t0
        progress(f"point cloud generated in {pc_gen:.1f} s")
        pct = [torch.from_numpy(a).to(dev) for a in (pc.points, pc.edges, pc.indptr, pc.indices, pc.data, pc.rhs)]
        pcx = torch.zeros_like(pct[5])
        pstats = {}

        def pc_step(form, tol, timed=None):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            h = build_hierarchy(*pct[:5], opt, stream)
            if timed is not None:
                torch.cuda.synchronize()
            tb = time.perf_counter()
            pcx.zero_()
            if form == "plain":
                _, inf, st = h.solve(pct[5], pcx, tol=tol, max_iters=400, stream=stream)
            else:
                _, inf, st = h.solve_pcg(pct[5], pcx, tol=tol, max_iters=200, precision="f32", stream=stream)
            if st != 0:
                raise RuntimeError(f"point cloud {form} solve did not converge (status {st})")
            if "sizes" not in pstats:
                pstats["sizes"] = [h.sizes(l) for l in range(h.num_levels)]
                pstats["levels"] = level_stats(h)
            h.free()
            torch.cuda.synchronize()
            tc = time.perf_counter()
            if timed is not None:
                timed.append((tb - ta, tc - tb))
            return inf
        ref_info = pc_step("plain", 1e-12)
        x_ref = pcx.cpu().numpy()
        pc_steps = max(2, min(args.steps, 5))
        legs = {}
        for form, tol in (("plain", args.tol), ("pcg_f32", 1e-10)):
            pc_step(form, tol)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(pc_steps):
                inf = pc_step(form, tol)
            torch.cuda.synchronize()
            fdt = (time.perf_counter() - t1) / pc_steps
            xs = pcx.cpu().numpy()
            parts = []
            for _ in range(2):
                pc_step(form, tol, parts)
            leg = {"value": 1.0 / fdt, "unit": "solves/s", "ms_per_step": 1e3 * fdt,
                   "setup_ms": 1e3 * min(p[0] for p in parts), "solve_ms": 1e3 * min(p[1] for p in parts),
                   "iterations": inf.iterations, "rel_residual": inf.rel_residual, "tol": tol,
                   "rel_error_vs_fp64_reference": float(np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref))}
            if form == "plain":
                psb = setup_bytes(pstats["sizes"])
                pcb = vcycle_bytes(pstats["sizes"], nu)
                pb_ = psb + inf.iterations * pcb
                leg["step_roofline"] = {"bytes": pb_, "achieved": pb_ / fdt / 1e9, "peak": 8000.0, "unit": "GB/s",
                                        "frac": pb_ / fdt / 8e12}
            legs[form] = leg
            progress(f"point cloud {form}: {leg['ms_per_step']:.1f} ms per step")
        pointcloud = {"workload": f"bumpy sphere point cloud, {pc.n} points, symmetrised kNN (k = 8) graph "
                                  f"({pc.m} edges), Gaussian graph Laplacian, (M + 1e-2 L) x = M b",
                      "generation_s": pc_gen, "plain_fp64": legs["plain"], "mixed_f32_cycle_fp64_cg": legs["pcg_f32"],
                      "fp64_reference": f"plain FP64 V-cycles to 1e-12 ({ref_info.iterations} cycles); the plain "
                                        "path's iterates are bit-identical to the CPU oracle's FP64 iterates",
                      "levels": pstats["levels"]}
        del pct, pcx

    out = {
        "metric": "setup+solve solves/s to 1e-8 rel. residual",
        "value": args.steps / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"torus {args.size}x{args.size} jittered, cotan (M + 1e-3 L) x = M b",
                   "points": prob.n, "edges": prob.m, "nnz_A": prob.nnz, "levels": levels,
                   "v_cycles": info.iterations, "rel_residual": info.rel_residual, "tol": args.tol},
        "roofline": lines[0] if lines else None,
        "roofline_other": lines[1:],
        "step_roofline": step_roofline,
        "levels": stats["levels"],
        "paper_fallback_pct": 0.25,
        "cpu_baseline": None,
        "mixed_vs_fp64": dict(forms, note="double CG preconditioned by one symmetric V-cycle per iteration "
                                          "(f64: cycle in double, f32: cycle in float); whole setup + solve "
                                          "per step, same workload and tolerance"),
        "split_ms": None if args.headline_only else {"plain": split("plain"), "pcg_f32": split("pcg_f32")},
        "pointcloud": pointcloud,
    }

    # many meshes of uneven size with 8 right-hand sides each: every hierarchy built and every
    # right-hand side solved to the same tolerance; batched float-preconditioned CG on concurrent
    # streams against the plain double V-cycle solve of each right-hand side in turn
    if not args.no_batched and not args.headline_only:
        out["batched"] = batched_leg(args, dev, opt)

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * src.numel() * 8

    if not args.no_cpu_baseline:
        import oracle
        progress("CPU oracle on one pinned core")

        def run_oracle():
            t0 = time.perf_counter()
            orc = oracle.Hierarchy.from_problem(prob)
            res = orc.solve(prob.rhs, tol=args.tol)
            return res, time.perf_counter() - t0
        ((xo, it, hist, st), cdt), core = pinned(run_oracle)
        err = float(np.linalg.norm(x_plain - xo) / np.linalg.norm(xo))
        for form, xf in x_forms.items():
            forms[form]["rel_error_vs_oracle_fp64"] = float(np.linalg.norm(xf - xo) / np.linalg.norm(xo))
        hc = host_cpu()
        out["cpu_baseline"] = {"value": 1.0 / cdt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full setup+solve of the same torus workload "
                                         f"({it} V-cycles, {cdt:.1f} s, single-threaded C++)",
                               "host": f"1 core of {hc['nproc']} ({hc['allowed_cores']} allowed to this "
                                       f"process), {hc['model']}",
                               "pinned_core": core, "nproc": hc["nproc"], "cpu_model": hc["model"],
                               "gpu_vs_oracle_rel_error": err,
                               "gpu_vs_oracle_bitwise": bool(np.array_equal(x_plain.view(np.int64),
                                                                            xo.view(np.int64)))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
