"""Many meshes at once.  Every mesh's hierarchy build runs on its own HIP
stream from a small pool of host threads, so that the latency-bound launches
of different meshes overlap on the device (a build waits for device scalars
between its steps; with several streams the device works on another mesh
meanwhile).  The solves then run either per mesh on the same streams, or as
one grouped CG over all hierarchies (gmg_solve_pcg_grouped: every step of an
iteration one launch for all meshes).  Every step runs through the C ABI;
this module only schedules.
"""
from concurrent.futures import ThreadPoolExecutor
import threading

from .binding import build_hierarchy, default_options, solve_pcg_grouped


def solve_many(systems, streams=4, tol=1e-8, max_iters=100, precision="f32", options=None, form="pcg",
               timing=None):
    """systems: list of (points, edges, rowptr, col, val, B) device tensors, B of shape
    (nrhs, n).  Returns a list of (X, infos, status) in the order of systems.

    form "pcg": the batched CG (gmg_solve_pcg_batched) in the given precision, per mesh;
    form "grouped": the same CG for all meshes at once (gmg_solve_pcg_grouped, at most
    8 right-hand sides per mesh), on the caller's stream after the builds;
    form "plain": the plain V-cycle solve (gmg_solve) of each right-hand side in
    turn, in double (the reference the batched form is compared with).
    timing: optional dict; the grouped form stores its build and solve seconds in it."""
    import torch
    opt = options if options is not None else default_options()
    local = threading.local()
    # the inputs may still be written by kernels on the caller's stream: every
    # worker stream waits for it before its first use of them
    caller = torch.cuda.current_stream()

    if form == "grouped":
        if any(int(a[5].shape[0]) > 8 for a in systems):
            raise ValueError("the grouped form takes at most 8 right-hand sides per mesh")

        def build(sysargs):
            points, edges, rowptr, col, val, _ = sysargs
            if not hasattr(local, "stream"):
                local.stream = torch.cuda.Stream()
            s = local.stream
            s.wait_stream(caller)
            with torch.cuda.stream(s):
                h = build_hierarchy(points, edges, rowptr, col, val, opt, s)
            s.synchronize()
            return h

        import time
        t0 = time.perf_counter()
        if streams <= 1:
            hs = [build(a) for a in systems]
        else:
            with ThreadPoolExecutor(max_workers=streams) as ex:
                hs = list(ex.map(build, systems))
        t1 = time.perf_counter()
        try:
            Xs, infos, sts, _ = solve_pcg_grouped(hs, [a[5] for a in systems], tol=tol, max_iters=max_iters,
                                                  precision=precision, stream=caller)
            if timing is not None:
                timing["build_s"] = t1 - t0
                timing["solve_s"] = time.perf_counter() - t1
        finally:
            for h in hs:
                h.free()
        return list(zip(Xs, infos, sts))

    def one(sysargs):
        points, edges, rowptr, col, val, B = sysargs
        if not hasattr(local, "stream"):
            local.stream = torch.cuda.Stream()
        s = local.stream
        s.wait_stream(caller)
        with torch.cuda.stream(s):
            h = build_hierarchy(points, edges, rowptr, col, val, opt, s)
            if form == "plain":
                X = torch.zeros_like(B)
                infos, st = [], 0
                for q in range(B.shape[0]):
                    _, info, stq = h.solve(B[q], X[q], tol=tol, max_iters=max_iters, stream=s)
                    infos.append(info)
                    st = st or stq
            else:
                X, infos, st = h.solve_pcg_batched(B, tol=tol, max_iters=max_iters, precision=precision,
                                                   stream=s)
            h.free()
        # X was allocated on s and is handed to the caller's stream: the caching
        # allocator must not reuse its block before the caller's work on it ends
        X.record_stream(caller)
        s.synchronize()
        return X, infos, st

    if streams <= 1:
        return [one(a) for a in systems]
    with ThreadPoolExecutor(max_workers=streams) as ex:
        return list(ex.map(one, systems))
