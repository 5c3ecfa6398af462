"""The seeded input generators: sizes, determinism and operator properties."""
import numpy as np
import scipy.sparse as sp

import synth
from tests.conftest import problem


def test_rng_is_splitmix64():
    # SplitMix64 seeded with the state key: value i is mix64(key + (i+1) * gamma)
    g = 0x9E3779B97F4A7C15
    key = int(synth.mix64([(0 + 2 * g) % 2**64])[0])           # seed 0, stream 1
    from synth.rng import raw64
    got = raw64(0, 1, 3)
    want = [int(synth.mix64([(key + (i + 1) * g) % 2**64])[0]) for i in range(3)]
    assert [int(v) for v in got] == want
    u = synth.uniform(0, "rhs", 100000, -1, 1)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01
    z = synth.normal(0, "jitter", 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


def test_icosphere_sizes():
    pts, faces = synth.icosphere(5)
    assert pts.shape == (10242, 3) and faces.shape == (20480, 3)
    assert synth.edges_from_faces(faces).shape == (30720, 2)
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0)


def test_torus_sizes():
    pts, faces = synth.torus_grid(32, 24)
    e = synth.edges_from_faces(faces)
    assert pts.shape == (768, 3) and faces.shape == (1536, 3) and e.shape == (3 * 768, 2)
    deg = np.bincount(e.ravel(), minlength=768)
    assert np.all(deg == 6)


def test_mesh_problem_is_spd_and_deterministic():
    a = problem("torus48")
    b = synth.small_torus(48, 40)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.data, b.data)
    A = a.matrix()
    assert abs(A - A.T).max() == 0
    assert np.all(np.diff(a.indptr) == 7)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    # pattern = edges plus diagonal
    rows = np.repeat(np.arange(a.n), np.diff(a.indptr))
    off = rows != a.indices
    assert off.sum() == 2 * a.m


def test_pointcloud_problem():
    p = problem("pc4k")
    A = p.matrix()
    assert abs(A - A.T).max() == 0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    deg = np.bincount(p.edges.ravel(), minlength=p.n)
    assert deg.min() >= 8
