"""Many meshes at once: every mesh's hierarchy build and batched solve runs
on its own HIP stream from a small pool of host threads, so that the
latency-bound launches of different meshes overlap on the device (a build or
a solve waits for device scalars between its steps; with several streams the
device works on another mesh meanwhile).  Every step runs through the C ABI;
this module only schedules.
"""
from concurrent.futures import ThreadPoolExecutor
import threading

from .binding import build_hierarchy, default_options


def solve_many(systems, streams=4, tol=1e-8, max_iters=100, precision="f32", options=None, form="pcg"):
    """systems: list of (points, edges, rowptr, col, val, B) device tensors, B of shape
    (nrhs, n).  Returns a list of (X, infos, status) in the order of systems.

    form "pcg": the batched CG (gmg_solve_pcg_batched) in the given precision;
    form "plain": the plain V-cycle solve (gmg_solve) of each right-hand side in
    turn, in double (the reference the batched form is compared with)."""
    import torch
    opt = options if options is not None else default_options()
    local = threading.local()
    # the inputs may still be written by kernels on the caller's stream: every
    # worker stream waits for it before its first use of them
    caller = torch.cuda.current_stream()

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
