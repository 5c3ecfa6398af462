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
# for a plain device copy (profiles/k_gs_color_*_torus1024.md); valid only for the kernel sources
# they were taken on (sha256 prefix of solve.hip + rows.hpp).
TRAFFIC = {"gs_finest": {"bytes_per_launch": 26822506, "src_sha256_16": "c193cd04f86734a6"},
           "gs_galerkin": {"bytes_per_launch": 2557707, "src_sha256_16": "c193cd04f86734a6"}}

KERNEL_NAMES = {"gs_finest": "k_gs_color_fine (one colour of a Gauss-Seidel sweep, level 0)",
                "residual_finest": "k_residual_norm (residual + norm partials, level 0)",
                "gs_galerkin": "k_gs_color<R> (one colour of a Gauss-Seidel sweep, Galerkin levels above the tail)"}


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("solve.hip", "rows.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2307_04886_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kind):
    rec = TRAFFIC.get(kind)
    if rec is None:
        return None
    return rec["bytes_per_launch"] if kernel_src_sha() == rec["src_sha256_16"] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-mesh batched measurement")
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
    x_plain = x.cpu().numpy()

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
        "cpu_baseline": None,
        "mixed_vs_fp64": dict(forms, note="double CG preconditioned by one symmetric V-cycle per iteration "
                                          "(f64: cycle in double, f32: cycle in float); whole setup + solve "
                                          "per step, same workload and tolerance"),
        "split_ms": None if args.headline_only else {"plain": split("plain"), "pcg_f32": split("pcg_f32")},
    }

    # many meshes of uneven size with 8 right-hand sides each: every hierarchy built and every
    # right-hand side solved to the same tolerance; batched float-preconditioned CG on concurrent
    # streams against the plain double V-cycle solve of each right-hand side in turn
    if not args.no_batched and not args.headline_only:
        from paper_2307_04886_amd.batch import solve_many
        batch = synth.config_batched()
        systems = []
        for bp, B in batch:
            t = [torch.from_numpy(a).to(dev) for a in (bp.points, bp.edges, bp.indptr, bp.indices, bp.data)]
            systems.append(tuple(t) + (torch.from_numpy(B).to(dev),))
        nsolves = sum(B.shape[0] for _, B in batch)
        solve_many(systems, streams=4, tol=args.tol, precision="f32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = solve_many(systems, streams=4, tol=args.tol, precision="f32")
        torch.cuda.synchronize()
        bdt = time.perf_counter() - t1
        if any(st != 0 for _, _, st in res):
            raise RuntimeError("batched solve did not converge")

        def plain_all():
            for (pts_, e_, rp_, ci_, va_, B) in systems:
                hh = build_hierarchy(pts_, e_, rp_, ci_, va_, opt, stream)
                for q in range(B.shape[0]):
                    xq = torch.zeros_like(B[q])
                    _, inf, st = hh.solve(B[q].contiguous(), xq, tol=args.tol, max_iters=200, stream=stream)
                    if st != 0:
                        raise RuntimeError("plain solve did not converge")
                hh.free()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_all()
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t1
        out["batched"] = {"workload": f"{len(batch)} jittered tori and icospheres, {min(b.n for b, _ in batch)}"
                                      f"-{max(b.n for b, _ in batch)} vertices ({sum(b.n for b, _ in batch)} in total),"
                                      f" 8 right-hand sides each, (M + 1e-3 L), tol {args.tol}",
                          "value": nsolves / bdt, "unit": "solves/s", "ms": 1e3 * bdt, "solves": nsolves,
                          "form": "setup + float-preconditioned double CG, 8 right-hand sides per launch, "
                                  "4 streams",
                          "plain_fp64_value": nsolves / pdt, "plain_fp64_ms": 1e3 * pdt,
                          "vs_plain_fp64": pdt / bdt}

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * src.numel() * 8

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        orc = oracle.Hierarchy.from_problem(prob)
        xo, it, hist, st = orc.solve(prob.rhs, tol=args.tol)
        cdt = time.perf_counter() - t0
        err = float(np.linalg.norm(x_plain - xo) / np.linalg.norm(xo))
        for form, xf in x_forms.items():
            forms[form]["rel_error_vs_oracle_fp64"] = float(np.linalg.norm(xf - xo) / np.linalg.norm(xo))
        out["cpu_baseline"] = {"value": 1.0 / cdt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full setup+solve of the same torus workload "
                                         f"({it} V-cycles, {cdt:.1f} s, single-threaded C++)",
                               "gpu_vs_oracle_rel_error": err}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
