"""The seeded generator: determinism, index ranges, one nonzero per (fascicle, voxel)."""
import numpy as np

import synth
from conftest import connectome


def test_tiny_deterministic_and_in_range():
    a = synth.make("tiny")
    b = synth.make("tiny")
    for k in ("atom", "voxel", "fascicle", "phi", "D", "w0", "w_true", "noise"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert a.n_theta == 16 and a.n_atoms == 64 and a.n_voxels == 512 and a.n_fascicles == 200
    assert 1000 <= a.nnz <= 4000
    assert a.atom.dtype == np.int16 and a.voxel.dtype == np.int32 and a.fascicle.dtype == np.int32
    assert a.atom.min() >= 0 and a.atom.max() < a.n_atoms
    assert a.voxel.min() >= 0 and a.voxel.max() < a.n_voxels
    assert a.fascicle.min() >= 0 and a.fascicle.max() < a.n_fascicles
    assert a.phi.min() >= 0.3 and a.phi.max() <= 1.2
    key = a.fascicle.astype(np.int64) * a.n_voxels + a.voxel
    assert np.unique(key).size == a.nnz
    # D columns are demeaned over theta
    assert np.abs(a.D.astype(np.float64).mean(axis=1)).max() < 1e-6


def test_mid_slice_shapes():
    c = connectome("mid", n_fascicles=20_000)
    assert c.n_theta == 96 and c.n_atoms == 1057
    assert 110_000 < c.n_voxels < 130_000
    assert c.atom.max() < 1057


def test_fibonacci_sphere_unit():
    u = synth.fibonacci_sphere(1057)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)
