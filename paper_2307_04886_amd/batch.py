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


def solve_many(systems, streams=4, tol=1e-8, max_iters=100, precision="f32", options=None):
    """systems: list of (points, edges, rowptr, col, val, B) device tensors, B of shape
    (nrhs, n).  Returns a list of (X, infos, status) in the order of systems."""
    import torch
    opt = options if options is not None else default_options()
    local = threading.local()

    def one(sysargs):
        points, edges, rowptr, col, val, B = sysargs
        if not hasattr(local, "stream"):
            local.stream = torch.cuda.Stream()
        s = local.stream
        with torch.cuda.stream(s):
            h = build_hierarchy(points, edges, rowptr, col, val, opt, s)
            X, infos, st = h.solve_pcg_batched(B, tol=tol, max_iters=max_iters, precision=precision, stream=s)
            h.free()
        s.synchronize()
        return X, infos, st

    if streams <= 1:
        return [one(a) for a in systems]
    with ThreadPoolExecutor(max_workers=streams) as ex:
        return list(ex.map(one, systems))
