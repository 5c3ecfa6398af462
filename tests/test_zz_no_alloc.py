"""GPU: gmg_precondition_noalloc (the preconditioner for callers that cannot
allocate device memory) against gmg_precondition through the C ABI: the same
kernels on a fixed scratch array, so z must be bit-identical, on two calls in
a row (the second on a smaller hierarchy, which finds the first call's values
in the shared scratch) and in both precisions."""
import sys

import numpy as np
import pytest

from tests.conftest import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _handle(name, minc):
    import paper_2307_04886_amd as g
    from paper_2307_04886_amd.binding import from_problem
    g.library()
    return from_problem(problem(name), g.default_options(min_coarse_points=minc))[0]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_matches_precondition(precision):
    _say(f"[gpu] gmg_precondition_noalloc {precision}: torus96, then the smaller ico4")
    big, small = _handle("torus96", 200), _handle("ico4", 100)
    assert small.n < big.n
    for k, h in enumerate((big, small)):
        r = torch.from_numpy(np.random.default_rng(40 + k).uniform(-1, 1, h.n)).cuda()
        ref = h.precondition(r, precision=precision)          # also makes the float level data
        z = torch.full_like(r, float("nan"))
        h.precondition_noalloc(r, z, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(z, ref), (k, precision)
        again = torch.full_like(r, float("nan"))
        h.precondition_noalloc(r, again, precision=precision)  # scratch now holds this handle's values
        torch.cuda.synchronize()
        assert torch.equal(again, ref), (k, precision)


def test_noalloc_rejects_what_it_cannot_do():
    _say("[gpu] gmg_precondition_noalloc errors")
    import paper_2307_04886_amd as g
    h = _handle("ico3", 100)
    r = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, h.n)).cuda()
    z = torch.zeros_like(r)
    with pytest.raises(g.GMGError) as e:                      # float data not made yet
        h.precondition_noalloc(r, z, precision="f32")
    assert e.value.status == -1
    h.precondition(r, precision="f32")
    h.precondition_noalloc(r, z, precision="f32")
    torch.cuda.synchronize()
    assert torch.equal(z, h.precondition(r, precision="f32"))
